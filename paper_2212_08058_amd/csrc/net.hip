// Warm-start network: four 'same' 3x3x3 convolutions (1 -> 16 -> 16 -> 16 -> 1
// channels, zero padding, bias, ReLU between layers) mapping the feature
// volume f to a start vector for the power iteration.
//
// Weights and activations are bfloat16, accumulation is FP32. Hidden
// activations are stored channels-last ([voxel][16], 32 bytes per voxel).
// The two 16 -> 16 layers, and their input gradients, run as implicit GEMMs on
// the matrix cores (v_mfma_f32_16x16x16_bf16): per wavefront a 16-channel x
// 16-voxel output block accumulates 27 taps of (16 out x 16 in) weights times
// (16 in x 16 voxels) inputs; so do their weight gradients (wgrad16_kernel,
// a sum over voxels of 16 x 16 outer products per tap). The 1 -> 16 and
// 16 -> 1 layers and their weight gradients are VALU kernels (their shapes fit
// the matrix cores badly).
//
// Parameter layout (FP32 masters, PyTorch conv3d order [Cout][Cin][3][3][3]):
//   w1[16][1][27] b1[16] w2[16][16][27] b2[16] w3[16][16][27] b3[16] w4[1][16][27] b4[1]
#include <hip/hip_runtime.h>

#include <algorithm>

#include <cmath>
#include <cstring>

#include "../../include/stpi.h"
#include "common.hpp"
#include "host_internal.hpp"

namespace stpi {

namespace net {

constexpr int C = 16;
constexpr int NT = 27;
constexpr int OFF_W1 = 0, OFF_B1 = 432, OFF_W2 = 448, OFF_B2 = 448 + 6912, OFF_W3 = OFF_B2 + 16,
              OFF_B3 = OFF_W3 + 6912, OFF_W4 = OFF_B3 + 16, OFF_B4 = OFF_W4 + 432, NPARAM = OFF_B4 + 1;
static_assert(NPARAM == 14737, "parameter count");

typedef short bf16x4 __attribute__((ext_vector_type(4)));
typedef float f32x4 __attribute__((ext_vector_type(4)));

// Prepared weights (device): rounded FP32 copies for the VALU layers and the
// per-lane MFMA operand blocks of the 16 -> 16 layers, forward and transposed/
// flipped (input gradient).
struct Prep {
    float w1[C][NT];       // [co][tap]
    float b1[C];
    bf16x4 a2[NT][64];     // forward A operand of layer 2: lane l -> W2[co=l%16][ci=4(l/16)+j][tap]
    bf16x4 a2d[NT][64];    // input-gradient A operand:     lane l -> W2[co=4(l/16)+j][ci=l%16][26-tap]
    float b2[C];
    bf16x4 a3[NT][64];
    bf16x4 a3d[NT][64];
    float b3[C];
    float w4[C][NT];       // [ci][tap]
    float b4;
};

__device__ __forceinline__ float bfr(float v) { return __uint_as_float(((uint32_t)f32_to_bf16_bits(v)) << 16); }
__device__ __forceinline__ short bfbits(float v) { return (short)f32_to_bf16_bits(v); }
__device__ __forceinline__ float bf2f(short b) { return __uint_as_float(((uint32_t)(uint16_t)b) << 16); }

__global__ void prepare_kernel(const float *m, Prep *p) {
    const int tid = blockIdx.x * blockDim.x + threadIdx.x;
    const int nth = gridDim.x * blockDim.x;
    for (int i = tid; i < C * NT; i += nth) {
        const int co = i / NT, tap = i % NT;
        p->w1[co][tap] = bfr(m[OFF_W1 + i]);
        p->w4[co][tap] = bfr(m[OFF_W4 + i]);  // w4[0][ci=co][tap]
    }
    for (int i = tid; i < NT * 64; i += nth) {
        const int tap = i / 64, l = i % 64;
        bf16x4 f2, d2, f3, d3;
        for (int j = 0; j < 4; ++j) {
            const int co = l % 16, ci = 4 * (l / 16) + j;          // forward
            f2[j] = bfbits(m[OFF_W2 + (co * C + ci) * NT + tap]);
            f3[j] = bfbits(m[OFF_W3 + (co * C + ci) * NT + tap]);
            const int co2 = 4 * (l / 16) + j, ci2 = l % 16;        // transposed, flipped
            d2[j] = bfbits(m[OFF_W2 + (co2 * C + ci2) * NT + (NT - 1 - tap)]);
            d3[j] = bfbits(m[OFF_W3 + (co2 * C + ci2) * NT + (NT - 1 - tap)]);
        }
        p->a2[tap][l] = f2;
        p->a2d[tap][l] = d2;
        p->a3[tap][l] = f3;
        p->a3d[tap][l] = d3;
    }
    if (tid < C) {
        p->b1[tid] = m[OFF_B1 + tid];
        p->b2[tid] = m[OFF_B2 + tid];
        p->b3[tid] = m[OFF_B3 + tid];
    }
    if (tid == 0) p->b4 = m[OFF_B4];
}

struct Dims {
    int T, H, W;
};

__device__ __forceinline__ bool inside(const Dims &d, int t, int y, int x) {
    return (unsigned)t < (unsigned)d.T && (unsigned)y < (unsigned)d.H && (unsigned)x < (unsigned)d.W;
}

// Raw buffer loads over a channels-last activation volume: an out-of-range
// byte offset reads 0, so the loads of the zero padding need no branch (and
// the compiler no full memory wait where branches join). The host limits
// activation volumes to 2^31 bytes.
constexpr uint32_t OOB_OFF = 0xFFFFFFF0u;
__device__ __forceinline__ __amdgpu_buffer_rsrc_t act_rsrc(const short *base, const Dims &d) {
    const int bytes = (int)((size_t)d.T * d.H * d.W * C * sizeof(short));
    return __builtin_amdgcn_make_buffer_rsrc(const_cast<short *>(base), (short)0, bytes, 0x00020000);
}
__device__ __forceinline__ bf16x4 load_b64(__amdgpu_buffer_rsrc_t r, uint32_t boff) {
    return __builtin_bit_cast(bf16x4, __builtin_amdgcn_raw_buffer_load_b64(r, boff, 0, 0));
}
__device__ __forceinline__ short load_b16(__amdgpu_buffer_rsrc_t r, uint32_t boff) {
    return (short)__builtin_amdgcn_raw_buffer_load_b16(r, boff, 0, 0);
}

typedef short bf16x8 __attribute__((ext_vector_type(8)));
typedef __bf16 bf16v8 __attribute__((ext_vector_type(8)));

// Layer 1 (1 -> 16), ReLU. f is FP32 and enters rounded to bfloat16. One
// v_mfma_f32_16x16x32_bf16 per 16 voxels of a row: A = W1 [co][tap] with the
// 27 taps padded to K = 32 (lane l holds co = l % 16, taps 8 (l / 16) .. + 7),
// B = the voxels' 27 neighbours (lane l: voxel l % 16, the same taps),
// gathered with buffer loads whose out-of-range offsets read the zero padding.
__global__ __launch_bounds__(256) void conv_in_kernel(Dims d, const float *f, const Prep *p, short *act) {
    const int lane = threadIdx.x & 63;
    const int wave = blockIdx.x * (blockDim.x / 64) + (threadIdx.x >> 6);
    const int nwaves = gridDim.x * (blockDim.x / 64);
    const int n = lane % 16, kq = lane / 16;
    bf16x8 aw;
#pragma unroll
    for (int j = 0; j < 8; ++j) {
        const int tap = 8 * kq + j;
        aw[j] = tap < NT ? bfbits(p->w1[n][tap]) : (short)0;  // the masters are already bfloat16 values
    }
    float bias[4];
#pragma unroll
    for (int j = 0; j < 4; ++j) bias[j] = p->b1[4 * kq + j];
    const int bytes = (int)((size_t)d.T * d.H * d.W * sizeof(float));
    const auto rf = __builtin_amdgcn_make_buffer_rsrc(const_cast<float *>(f), (short)0, bytes, 0x00020000);
    const int gx = (d.W + 15) / 16;
    const int ngroups = d.T * d.H * gx;
    constexpr int GB = 4;  // groups whose gathers are in flight together
    for (int g0 = wave * GB; g0 < ngroups; g0 += nwaves * GB) {
        bf16x8 bv[GB];
#pragma unroll
        for (int h = 0; h < GB; ++h) {
            const int g = g0 + h < ngroups ? g0 + h : ngroups - 1;
            const int xg = g % gx, y = (g / gx) % d.H, t = g / (gx * d.H);
            const int x = xg * 16 + n;
#pragma unroll
            for (int j = 0; j < 8; ++j) {
                const int tap = 8 * kq + j;
                const int tt = t + tap / 9 - 1, yy = y + (tap / 3) % 3 - 1, xx = x + tap % 3 - 1;
                const bool ok = tap < NT && inside(d, tt, yy, xx);
                const uint32_t off = (uint32_t)(((size_t)tt * d.H + yy) * d.W + xx) * 4;
                bv[h][j] = bfbits(__uint_as_float(__builtin_amdgcn_raw_buffer_load_b32(rf, ok ? off : OOB_OFF, 0, 0)));
            }
        }
#pragma unroll
        for (int h = 0; h < GB; ++h) {
            const int g = g0 + h;
            if (g >= ngroups) break;
            const int xg = g % gx, y = (g / gx) % d.H, t = g / (gx * d.H);
            const int x = xg * 16 + n;
            f32x4 acc = __builtin_amdgcn_mfma_f32_16x16x32_bf16(__builtin_bit_cast(bf16v8, aw),
                                                                __builtin_bit_cast(bf16v8, bv[h]),
                                                                f32x4{0.f, 0.f, 0.f, 0.f}, 0, 0, 0);
            // lane holds pre-activation[co = 4 kq + j][voxel n]
            if (x < d.W) {
                const size_t v = ((size_t)t * d.H + y) * d.W + x;
                bf16x4 o;
#pragma unroll
                for (int j = 0; j < 4; ++j) o[j] = bfbits(fmaxf(acc[j] + bias[j], 0.0f));
                *reinterpret_cast<bf16x4 *>(act + v * C + 4 * kq) = o;
            }
        }
    }
}

// Lane n of each 16-lane row takes src from lane n + 1 (ROW_SHL1) or n - 1
// (ROW_SHR1) of the same row; lanes whose source lies outside the row keep
// `old` (the neighbouring tile's edge voxel).
constexpr int DPP_ROW_SHL1 = 0x101, DPP_ROW_SHR1 = 0x111;
template <int CTRL>
__device__ __forceinline__ bf16x4 row_shift(bf16x4 src, bf16x4 old) {
    union U {
        bf16x4 v;
        int i[2];
    } s, o, r;
    s.v = src;
    o.v = old;
    r.i[0] = __builtin_amdgcn_update_dpp(o.i[0], s.i[0], CTRL, 0xF, 0xF, false);
    r.i[1] = __builtin_amdgcn_update_dpp(o.i[1], s.i[1], CTRL, 0xF, 0xF, false);
    return r.v;
}

constexpr int CONV_RB = 4;  // output rows per wavefront

// 16 -> 16 convolution on the matrix cores. mode 0: out = relu(conv + bias);
// mode 1 (input gradient of a ReLU layer): out = conv(g, flipped W^T) masked
// by mask > 0. One wavefront per 16 consecutive voxels of CONV_RB rows: each
// input row (per frame offset) is loaded once, as 16 voxels plus the two edge
// voxels (one load: lane 0 takes x0 - 1, lane 15 x0 + 16), and feeds up to
// three output rows; the x-1 and x+1 taps take the
// row's registers shifted by one lane (DPP), so every activation is read
// from memory about (CONV_RB + 2) / CONV_RB * 3 times instead of 27. A
// group's 3 (CONV_RB + 2) row loads are all issued before its MFMAs.
template <int MODE>
__global__ __launch_bounds__(256, 3) void conv16_kernel(Dims d, const short *in, const bf16x4 (*A)[64],
                                                     const float *bias, const short *mask, short *out) {
    const int lane = threadIdx.x & 63;
    const int wave = blockIdx.x * (blockDim.x / 64) + (threadIdx.x >> 6);
    const int gx = (d.W + 15) / 16, gy = (d.H + CONV_RB - 1) / CONV_RB;
    const int ngroups = d.T * gy * gx;
    const int nwaves = gridDim.x * (blockDim.x / 64);
    const int n = lane % 16, kq = lane / 16;  // voxel column of B, channel quad
    const auto rs = act_rsrc(in, d);
    bf16x4 a[NT];
#pragma unroll
    for (int tap = 0; tap < NT; ++tap) a[tap] = A[tap][lane];
    for (int g = wave; g < ngroups; g += nwaves) {
        const int xg = g % gx, yb = (g / gx) % gy, t = g / (gx * gy);
        const int x0 = xg * 16, y0 = yb * CONV_RB, x = x0 + n;
        f32x4 acc[CONV_RB];
#pragma unroll
        for (int r = 0; r < CONV_RB; ++r) acc[r] = f32x4{0.f, 0.f, 0.f, 0.f};
        // all the group's input rows are loaded first (rows and frames outside
        // the volume read as zero), so their latencies overlap
        constexpr int NR = 3 * (CONV_RB + 2);
        // b0: the lane's voxel; be: the row's edge voxel the shifts bring in
        // (x0 - 1 for lane 0, x0 + 16 for lane 15; other lanes never use it)
        const int xe = n == 0 ? x0 - 1 : x0 + 16;
        const bool eok = xe >= 0 && xe < d.W;
        bf16x4 b0[NR], be[NR];
#pragma unroll
        for (int k = 0; k < NR; ++k) {
            const int tt = t + k / (CONV_RB + 2) - 1, yy = y0 - 1 + k % (CONV_RB + 2);
            const bool rowok = tt >= 0 && tt < d.T && yy >= 0 && yy < d.H;
            const uint32_t row = (uint32_t)(((size_t)tt * d.H + yy) * d.W) * (C * 2) + 8 * kq;
            b0[k] = load_b64(rs, rowok && x < d.W ? row + (uint32_t)x * (C * 2) : OOB_OFF);
            be[k] = load_b64(rs, rowok && eok ? row + (uint32_t)xe * (C * 2) : OOB_OFF);
        }
#pragma unroll
        for (int k = 0; k < NR; ++k) {
            const int dt = k / (CONV_RB + 2) - 1, ry = k % (CONV_RB + 2);
            const bf16x4 bl = row_shift<DPP_ROW_SHR1>(b0[k], be[k]);  // voxel x - 1 (lane 0 keeps be)
            const bf16x4 br = row_shift<DPP_ROW_SHL1>(b0[k], be[k]);  // voxel x + 1 (lane 15 keeps be)
#pragma unroll
            for (int dy = -1; dy <= 1; ++dy) {
                const int r = ry - 1 - dy;  // output row fed by this input row through dy
                if (r < 0 || r >= CONV_RB) continue;
                const int tap = (dt + 1) * 9 + (dy + 1) * 3;
                acc[r] = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(a[tap], bl, acc[r], 0, 0, 0);
                acc[r] = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(a[tap + 1], b0[k], acc[r], 0, 0, 0);
                acc[r] = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(a[tap + 2], br, acc[r], 0, 0, 0);
            }
        }
        // lane holds out[co = 4 kq + j][voxel n] of each row
#pragma unroll
        for (int r = 0; r < CONV_RB; ++r) {
            const int y = y0 + r;
            if (y >= d.H || x >= d.W) continue;
            const size_t v = ((size_t)t * d.H + y) * d.W + x;
            bf16x4 o;
            if (MODE == 0) {
#pragma unroll
                for (int j = 0; j < 4; ++j) o[j] = bfbits(fmaxf(acc[r][j] + bias[4 * kq + j], 0.0f));
            } else {
                const bf16x4 mk = *reinterpret_cast<const bf16x4 *>(mask + v * C + 4 * kq);
#pragma unroll
                for (int j = 0; j < 4; ++j) o[j] = bf2f(mk[j]) > 0.0f ? bfbits(acc[r][j]) : (short)0;
            }
            *reinterpret_cast<bf16x4 *>(out + v * C + 4 * kq) = o;
        }
    }
}

// Layer 4 (16 -> 1), no activation: y = b4 + sum w4 * act3.
__global__ __launch_bounds__(256) void conv_out_kernel(Dims d, const short *act, const Prep *p, float *y) {
    __shared__ float w[C][NT];
    for (int i = threadIdx.x; i < C * NT; i += blockDim.x) w[i / NT][i % NT] = p->w4[i / NT][i % NT];
    __syncthreads();
    const float b4 = p->b4;
    const size_t V = (size_t)d.T * d.H * d.W;
    for (size_t v = (size_t)blockIdx.x * blockDim.x + threadIdx.x; v < V; v += (size_t)gridDim.x * blockDim.x) {
        const int x = (int)(v % d.W), yy0 = (int)((v / d.W) % d.H), t = (int)(v / ((size_t)d.W * d.H));
        float s = b4;
        for (int tap = 0; tap < NT; ++tap) {
            const int tt = t + tap / 9 - 1, yy = yy0 + (tap / 3) % 3 - 1, xx = x + tap % 3 - 1;
            if (!inside(d, tt, yy, xx)) continue;
            const bf16x4 *src = reinterpret_cast<const bf16x4 *>(act + (((size_t)tt * d.H + yy) * d.W + xx) * C);
#pragma unroll
            for (int q = 0; q < 4; ++q) {
                const bf16x4 a = src[q];
#pragma unroll
                for (int j = 0; j < 4; ++j) s = fmaf(w[4 * q + j][tap], bf2f(a[j]), s);
            }
        }
        y[v] = s;
    }
}

// Loss MSE(y, x* sqrt(V)) and g_y = 2 (y - x* sqrt(V)) / V; partials[2b] = sum of squares.
__global__ void mse_kernel(size_t V, const float *y, const float *xs, double scale, float *gy, double *partials) {
    __shared__ double red[256 / 64];
    double s = 0.0;
    const double inv = 1.0 / (double)V;
    for (size_t v = (size_t)blockIdx.x * 256 + threadIdx.x; v < V; v += (size_t)gridDim.x * 256) {
        const double dlt = (double)y[v] - (double)xs[v] * scale;
        s += dlt * dlt;
        gy[v] = (float)(2.0 * dlt * inv);
    }
    const double t = block_sum<256>(s, red);
    if (threadIdx.x == 0) {
        partials[2 * blockIdx.x] = t;
        partials[2 * blockIdx.x + 1] = 0.0;
    }
}

__global__ __launch_bounds__(256) void mse_finalize(int nb, size_t V, const double *partials, double *loss) {
    __shared__ double red[256 / 64];
    double s = 0.0;
    for (int b = threadIdx.x; b < nb; b += 256) s += partials[2 * b];
    s = block_sum<256>(s, red);
    if (threadIdx.x == 0) *loss = s / (double)V;
}

// Input gradient of layer 4, masked by layer 3's ReLU:
// g3[v][ci] = (act3[v][ci] > 0) * sum_tap w4[ci][tap] * g_y[v - tap]
__global__ __launch_bounds__(256) void out_bwd_kernel(Dims d, const float *gy, const short *act3, const Prep *p, short *g3) {
    __shared__ float w[C][NT];
    for (int i = threadIdx.x; i < C * NT; i += blockDim.x) w[i / NT][i % NT] = p->w4[i / NT][i % NT];
    __syncthreads();
    const size_t V = (size_t)d.T * d.H * d.W;
    for (size_t v = (size_t)blockIdx.x * blockDim.x + threadIdx.x; v < V; v += (size_t)gridDim.x * blockDim.x) {
        const int x = (int)(v % d.W), y = (int)((v / d.W) % d.H), t = (int)(v / ((size_t)d.W * d.H));
        float g[NT];
#pragma unroll
        for (int tap = 0; tap < NT; ++tap) {
            const int tt = t - (tap / 9 - 1), yy = y - ((tap / 3) % 3 - 1), xx = x - (tap % 3 - 1);
            g[tap] = inside(d, tt, yy, xx) ? gy[((size_t)tt * d.H + yy) * d.W + xx] : 0.0f;
        }
        const bf16x4 *ap = reinterpret_cast<const bf16x4 *>(act3 + v * C);
        bf16x4 *dst = reinterpret_cast<bf16x4 *>(g3 + v * C);
#pragma unroll
        for (int q = 0; q < 4; ++q) {
            const bf16x4 a = ap[q];
            bf16x4 o;
#pragma unroll
            for (int j = 0; j < 4; ++j) {
                float s = 0.0f;
#pragma unroll
                for (int tap = 0; tap < NT; ++tap) s = fmaf(w[4 * q + j][tap], g[tap], s);
                o[j] = bf2f(a[j]) > 0.0f ? bfbits(s) : (short)0;
            }
            dst[q] = o;
        }
    }
}


// Weight and bias gradients of a 16 -> 16 layer on the matrix cores. For each
// tap, dW_tap[co][ci] = sum_v g[v][co] a[v + tap][ci] is a (16 x V) x (V x 16)
// product: v_mfma_f32_16x16x4f32 takes 4 voxels per instruction, lane l
// holding g[v0 + l/16][co = l%16] (A) and a[v0 + l/16 + tap][ci = l%16] (B),
// so a wavefront's loads are contiguous runs of the channels-last volumes.
// Operands are the stored bfloat16 values widened exactly to float, so the
// products and FP32 sums are those of a bfloat16 matrix product with FP32
// accumulation. Each workgroup writes its partial sums ([co][ci * 27 + tap],
// then the bias of co); wgrad_reduce sums them.
__global__ __launch_bounds__(256, 2) void wgrad16_kernel(Dims d, const short *a, const short *g, float *partials) {
    constexpr int NP = C * (C * NT + 1);
    __shared__ float red[NP];
    const int lane = threadIdx.x & 63;
    const int wid = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    const int wave = blockIdx.x * 4 + wid;
    const int nwaves = gridDim.x * 4;
    const int ch = lane % 16, kv = lane / 16;
    const size_t V = (size_t)d.T * d.H * d.W;
    const size_t nq = (V + 3) / 4;
    const auto ra = act_rsrc(a, d), rg = act_rsrc(g, d);
    f32x4 acc[NT];
#pragma unroll
    for (int tap = 0; tap < NT; ++tap) acc[tap] = f32x4{0.f, 0.f, 0.f, 0.f};
    float bacc = 0.0f;
    // two quads of voxels per pass: their 56 loads are in flight together
    for (size_t q0 = (size_t)wave * 2; q0 < nq; q0 += (size_t)nwaves * 2) {
        float gv[2], av[2][NT];
#pragma unroll
        for (int h = 0; h < 2; ++h) {
            const size_t v = (q0 + h) * 4 + kv;
            const bool vin = v < V;
            const int x = vin ? (int)(v % d.W) : 0, y = vin ? (int)((v / d.W) % d.H) : 0;
            const int t = vin ? (int)(v / ((size_t)d.W * d.H)) : 0;
            gv[h] = bf2f(load_b16(rg, vin ? (uint32_t)(v * C + ch) * 2 : OOB_OFF));
#pragma unroll
            for (int tap = 0; tap < NT; ++tap) {
                const int tt = t + tap / 9 - 1, yy = y + (tap / 3) % 3 - 1, xx = x + tap % 3 - 1;
                const uint32_t off = (uint32_t)((((size_t)tt * d.H + yy) * d.W + xx) * C + ch) * 2;
                av[h][tap] = bf2f(load_b16(ra, vin && inside(d, tt, yy, xx) ? off : OOB_OFF));
            }
        }
#pragma unroll
        for (int h = 0; h < 2; ++h) {
            bacc += gv[h];
#pragma unroll
            for (int tap = 0; tap < NT; ++tap)
                acc[tap] = __builtin_amdgcn_mfma_f32_16x16x4f32(gv[h], av[h][tap], acc[tap], 0, 0, 0);
        }
    }
    // bias: lanes ch, ch + 16, ch + 32, ch + 48 hold the four voxel rows of channel ch
    float b = bacc + __shfl_xor(bacc, 16, 64);
    b += __shfl_xor(b, 32, 64);
    // the workgroup's four wavefronts add into LDS in turn (lane holds
    // dW_tap[co = 4 kv + j][ci = ch]), then one partial per workgroup
    for (int w = 0; w < 4; ++w) {
        if (wid == w) {
#pragma unroll
            for (int tap = 0; tap < NT; ++tap)
#pragma unroll
                for (int j = 0; j < 4; ++j) {
                    const int k = (4 * kv + j) * (C * NT + 1) + ch * NT + tap;
                    red[k] = (w == 0 ? 0.0f : red[k]) + acc[tap][j];
                }
            if (kv == 0) {
                const int k = ch * (C * NT + 1) + C * NT;
                red[k] = (w == 0 ? 0.0f : red[k]) + b;
            }
        }
        __syncthreads();
    }
    float *out = partials + (size_t)blockIdx.x * NP;
    for (int k = threadIdx.x; k < NP; k += 256) out[k] = red[k];
}

// Weight and bias gradients of the one-channel layers on the matrix cores
// (v_mfma_f32_16x16x4f32, four voxels per instruction, taps in two blocks of
// 16 columns):
//   MODE 1 (layer 1): D[co][tap] = sum_v g[v][co] bf16(f[v + off(tap)]),
//                     db1[co] = sum_v g[v][co]; X = g (channels-last), Z = f;
//   MODE 4 (layer 4): D[ci][tap] = sum_u act3[u][ci] g_y[u - off(tap)]
//                     (the same sum as over v = u - off), db4 = sum_v g_y[v];
//                     X = act3, Z = g_y.
// Lane l holds X[voxel l / 16][channel l % 16] (A operand) and Z at that
// voxel shifted by tap 16 blk + l % 16 (B operand); terms whose shifted voxel
// lies outside the volume read zero through out-of-range buffer offsets.
// Partial sums per workgroup: [co][ci * 27 + tap] then the bias of co (CI x 27 + 1 per co).
template <int MODE>
__global__ __launch_bounds__(256, 2) void wgrad1_kernel(Dims d, const short *x16, const float *z1, float *partials) {
    constexpr int NPR = MODE == 1 ? C * (NT + 1) : C * NT + 1;
    __shared__ float red[NPR];
    const int lane = threadIdx.x & 63;
    const int wid = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    const int wave = blockIdx.x * 4 + wid;
    const int nwaves = gridDim.x * 4;
    const int c = lane % 16, kv = lane / 16;
    const size_t V = (size_t)d.T * d.H * d.W;
    const size_t nq = (V + 3) / 4;
    const auto rx = act_rsrc(x16, d);
    const auto rz = __builtin_amdgcn_make_buffer_rsrc(const_cast<float *>(z1), (short)0, (int)(V * sizeof(float)),
                                                      0x00020000);
    int sdt[2], sdy[2], sdx[2];
    bool tapok[2];
#pragma unroll
    for (int blk = 0; blk < 2; ++blk) {
        const int tap = 16 * blk + c;
        tapok[blk] = tap < NT;
        const int s = MODE == 1 ? 1 : -1;  // layer 4 reads Z at u - off
        sdt[blk] = s * (tap / 9 - 1);
        sdy[blk] = s * ((tap / 3) % 3 - 1);
        sdx[blk] = s * (tap % 3 - 1);
    }
    f32x4 acc[2] = {f32x4{0.f, 0.f, 0.f, 0.f}, f32x4{0.f, 0.f, 0.f, 0.f}};
    float bacc = 0.0f;
    for (size_t q0 = (size_t)wave * 2; q0 < nq; q0 += (size_t)nwaves * 2) {
        float xa[2], zb[2][2];
#pragma unroll
        for (int h = 0; h < 2; ++h) {
            const size_t v = (q0 + h) * 4 + kv;
            const bool vin = v < V;
            const int x = vin ? (int)(v % d.W) : 0, y = vin ? (int)((v / d.W) % d.H) : 0;
            const int t = vin ? (int)(v / ((size_t)d.W * d.H)) : 0;
            xa[h] = bf2f(load_b16(rx, vin ? (uint32_t)(v * C + c) * 2 : OOB_OFF));
#pragma unroll
            for (int blk = 0; blk < 2; ++blk) {
                const int tt = t + sdt[blk], yy = y + sdy[blk], xx = x + sdx[blk];
                const bool ok = vin && tapok[blk] && inside(d, tt, yy, xx);
                const uint32_t off = (uint32_t)(((size_t)tt * d.H + yy) * d.W + xx) * 4;
                const float zv = __uint_as_float(__builtin_amdgcn_raw_buffer_load_b32(rz, ok ? off : OOB_OFF, 0, 0));
                zb[h][blk] = MODE == 1 ? bfr(zv) : zv;
            }
        }
#pragma unroll
        for (int h = 0; h < 2; ++h) {
            bacc += MODE == 1 ? xa[h] : (c == 13 ? zb[h][0] : 0.0f);  // tap 13 is the centre
#pragma unroll
            for (int blk = 0; blk < 2; ++blk)
                acc[blk] = __builtin_amdgcn_mfma_f32_16x16x4f32(xa[h], zb[h][blk], acc[blk], 0, 0, 0);
        }
    }
    // bias over the four voxel rows: lanes c, c + 16, c + 32, c + 48
    float b = bacc + __shfl_xor(bacc, 16, 64);
    b += __shfl_xor(b, 32, 64);
    // lane holds D[channel 4 kv + j][tap 16 blk + c]; the four wavefronts add into LDS in turn
    for (int w = 0; w < 4; ++w) {
        if (wid == w) {
#pragma unroll
            for (int blk = 0; blk < 2; ++blk)
#pragma unroll
                for (int j = 0; j < 4; ++j) {
                    if (!tapok[blk]) continue;
                    const int ch = 4 * kv + j, tap = 16 * blk + c;
                    const int k = MODE == 1 ? ch * (NT + 1) + tap : ch * NT + tap;
                    red[k] = (w == 0 ? 0.0f : red[k]) + acc[blk][j];
                }
            if (kv == 0 && (MODE == 1 || c == 13)) {
                const int k = MODE == 1 ? c * (NT + 1) + NT : C * NT;
                red[k] = (w == 0 ? 0.0f : red[k]) + b;
            }
        }
        __syncthreads();
    }
    float *out = partials + (size_t)blockIdx.x * NPR;
    for (int k = threadIdx.x; k < NPR; k += 256) out[k] = red[k];
}

constexpr int WG16_BLOCKS = 512;  // x 4 wavefronts (two per SIMD): one partial per workgroup

// Sums the workgroup partials of one layer into the gradient buffer (same
// layout as the masters): dW[co][ci][tap] at w_off, db[co] at b_off. One
// workgroup per entry: threads add strided partials in double, then the
// fixed block tree.
template <int CI, int CO>
__global__ __launch_bounds__(256) void wgrad_reduce(int nblocks, const float *partials, float *grad, int w_off,
                                                    int b_off) {
    constexpr int NP = CO * (CI * NT + 1);
    __shared__ double red[256 / 64];
    const int i = blockIdx.x;
    double s = 0.0;
    for (int b = threadIdx.x; b < nblocks; b += 256) s += (double)partials[(size_t)b * NP + i];
    s = block_sum<256>(s, red);
    if (threadIdx.x == 0) {
        const int co = i / (CI * NT + 1), r = i % (CI * NT + 1);
        if (r < CI * NT)
            grad[w_off + co * CI * NT + r] = (float)s;
        else
            grad[b_off + co] = (float)s;
    }
}

// Start vector from the net output: x0 = max(y, 0) + eps (normalised by the iteration).
__global__ void warm_x0_kernel(size_t V, const float *y, float eps, float *x0) {
    for (size_t v = (size_t)blockIdx.x * blockDim.x + threadIdx.x; v < V; v += (size_t)gridDim.x * blockDim.x)
        x0[v] = fmaxf(y[v], 0.0f) + eps;
}

constexpr int WG1_BLOCKS = 2048;  // x 4 wavefronts: wgrad1_kernel's partial sums (448 floats each)

}  // namespace net

}  // namespace stpi

using namespace stpi;
using namespace stpi::net;

extern "C" {

int stpi_net_param_count(void) { return NPARAM; }

size_t stpi_net_prep_bytes(void) { return sizeof(Prep); }

size_t stpi_net_workspace_bytes(const stpi_problem *p) {
    if (validate_problem(p) != STPI_OK) return 0;
    const size_t V = (size_t)p->T * p->H * p->W;
    // 3 activation volumes + 2 gradient volumes (bf16 x 16 channels), g_y, loss partials,
    // weight-gradient partials.
    size_t b = 5 * ((V * C * 2 + 255) & ~(size_t)255);
    b += (V * 4 + 255) & ~(size_t)255;
    b += 4096 * 8;
    b += std::max((size_t)WG1_BLOCKS * C * (NT + 1), (size_t)WG16_BLOCKS * C * (C * NT + 1)) * sizeof(float);
    return b;
}

int stpi_net_prepare(const float *master, void *prep, void *stream) {
    clear_error();
    if (!master || !prep) return fail(STPI_EINVAL, "NULL buffer");
    hipLaunchKernelGGL(prepare_kernel, dim3(8), dim3(256), 0, (hipStream_t)stream, master, (Prep *)prep);
    hipError_t e = hipGetLastError();
    return e == hipSuccess ? STPI_OK : hip_fail(e, "net prepare");
}

static int net_check(const stpi_problem *p, const void *ws, size_t ws_bytes) {
    int rc = validate_problem(p);
    if (rc) return rc;
    if ((size_t)p->T * p->H * p->W * C * sizeof(short) >= ((size_t)1 << 31))
        return fail(STPI_EUNSUPPORTED, "net volumes are limited to 2^31 bytes of activations (%d x %d x %d)", p->T,
                    p->H, p->W);
    if (!ws || ws_bytes < stpi_net_workspace_bytes(p))
        return fail(STPI_EWORKSPACE, "net workspace needs %zu bytes", stpi_net_workspace_bytes(p));
    return STPI_OK;
}

struct NetWs {
    short *act1, *act2, *act3, *g_a, *g_b;
    float *gy;
    double *lpart;
    float *wpart;
};

static NetWs net_ws(const stpi_problem *p, void *ws) {
    const size_t V = (size_t)p->T * p->H * p->W;
    const size_t vb = (V * C * 2 + 255) & ~(size_t)255;
    char *w = (char *)ws;
    NetWs n;
    n.act1 = (short *)w;
    n.act2 = (short *)(w + vb);
    n.act3 = (short *)(w + 2 * vb);
    n.g_a = (short *)(w + 3 * vb);
    n.g_b = (short *)(w + 4 * vb);
    char *q = w + 5 * vb;
    n.gy = (float *)q;
    q += (V * 4 + 255) & ~(size_t)255;
    n.lpart = (double *)q;
    q += 4096 * 8;
    n.wpart = (float *)q;
    return n;
}

static int conv16_grid(const stpi_problem *p) {
    const long groups = (long)p->T * ((p->H + CONV_RB - 1) / CONV_RB) * ((p->W + 15) / 16);
    const long blocks = (groups + 3) / 4;
    return (int)(blocks < 8192 ? blocks : 8192);
}

int stpi_net_forward(const stpi_problem *p, const float *f, const void *prep, float *y, void *ws, size_t ws_bytes,
                     void *stream) {
    clear_error();
    int rc = net_check(p, ws, ws_bytes);
    if (rc) return rc;
    if (!f || !prep || !y) return fail(STPI_EINVAL, "NULL buffer");
    const Prep *P = (const Prep *)prep;
    NetWs n = net_ws(p, ws);
    hipStream_t s = (hipStream_t)stream;
    const Dims d{p->T, p->H, p->W};
    hipLaunchKernelGGL(conv_in_kernel, dim3(conv16_grid(p)), dim3(256), 0, s, d, f, P, n.act1);
    hipLaunchKernelGGL(conv16_kernel<0>, dim3(conv16_grid(p)), dim3(256), 0, s, d, n.act1, P->a2, P->b2,
                       (const short *)nullptr, n.act2);
    hipLaunchKernelGGL(conv16_kernel<0>, dim3(conv16_grid(p)), dim3(256), 0, s, d, n.act2, P->a3, P->b3,
                       (const short *)nullptr, n.act3);
    hipLaunchKernelGGL(conv_out_kernel, dim3(2048), dim3(256), 0, s, d, n.act3, P, y);
    hipError_t e = hipGetLastError();
    return e == hipSuccess ? STPI_OK : hip_fail(e, "net forward");
}

int stpi_net_backward(const stpi_problem *p, const float *f, const void *prep, const float *y, const float *x_star,
                      double *loss, float *grad, void *ws, size_t ws_bytes, void *stream) {
    clear_error();
    int rc = net_check(p, ws, ws_bytes);
    if (rc) return rc;
    if (!f || !prep || !y || !x_star || !loss || !grad) return fail(STPI_EINVAL, "NULL buffer");
    const Prep *P = (const Prep *)prep;
    NetWs n = net_ws(p, ws);
    hipStream_t s = (hipStream_t)stream;
    const Dims d{p->T, p->H, p->W};
    const size_t V = (size_t)p->T * p->H * p->W;
    hipLaunchKernelGGL(mse_kernel, dim3(2048), dim3(256), 0, s, V, y, x_star, std::sqrt((double)V), n.gy, n.lpart);
    hipLaunchKernelGGL(mse_finalize, dim3(1), dim3(256), 0, s, 2048, V, n.lpart, loss);
    // layer 4
    hipLaunchKernelGGL(wgrad1_kernel<4>, dim3(WG1_BLOCKS), dim3(256), 0, s, d, (const short *)n.act3,
                       (const float *)n.gy, n.wpart);
    hipLaunchKernelGGL((wgrad_reduce<C, 1>), dim3(C * NT + 1), dim3(256), 0, s, WG1_BLOCKS, n.wpart, grad, OFF_W4, OFF_B4);
    hipLaunchKernelGGL(out_bwd_kernel, dim3(2048), dim3(256), 0, s, d, n.gy, n.act3, P, n.g_a);  // g at pre3
    // layer 3
    hipLaunchKernelGGL(wgrad16_kernel, dim3(WG16_BLOCKS), dim3(256), 0, s, d, (const short *)n.act2, n.g_a,
                       n.wpart);
    hipLaunchKernelGGL((wgrad_reduce<C, C>), dim3(C * (C * NT + 1)), dim3(256), 0, s,
                       WG16_BLOCKS, n.wpart, grad, OFF_W3, OFF_B3);
    hipLaunchKernelGGL(conv16_kernel<1>, dim3(conv16_grid(p)), dim3(256), 0, s, d, n.g_a, P->a3d,
                       (const float *)nullptr, n.act2, n.g_b);  // g at pre2
    // layer 2
    hipLaunchKernelGGL(wgrad16_kernel, dim3(WG16_BLOCKS), dim3(256), 0, s, d, (const short *)n.act1, n.g_b,
                       n.wpart);
    hipLaunchKernelGGL((wgrad_reduce<C, C>), dim3(C * (C * NT + 1)), dim3(256), 0, s,
                       WG16_BLOCKS, n.wpart, grad, OFF_W2, OFF_B2);
    hipLaunchKernelGGL(conv16_kernel<1>, dim3(conv16_grid(p)), dim3(256), 0, s, d, n.g_b, P->a2d,
                       (const float *)nullptr, n.act1, n.g_a);  // g at pre1
    // layer 1
    hipLaunchKernelGGL(wgrad1_kernel<1>, dim3(WG1_BLOCKS), dim3(256), 0, s, d, (const short *)n.g_a, f, n.wpart);
    hipLaunchKernelGGL((wgrad_reduce<1, C>), dim3(C * (NT + 1)), dim3(256), 0, s, WG1_BLOCKS, n.wpart, grad, OFF_W1, OFF_B1);
    hipError_t e = hipGetLastError();
    return e == hipSuccess ? STPI_OK : hip_fail(e, "net backward");
}

int stpi_net_warm_start(int64_t n, const float *y, float eps, float *x0, void *stream) {
    clear_error();
    if (n < 1 || !y || !x0) return fail(STPI_EINVAL, "bad arguments");
    hipLaunchKernelGGL(warm_x0_kernel, dim3(1024), dim3(256), 0, (hipStream_t)stream, (size_t)n, y, eps, x0);
    hipError_t e = hipGetLastError();
    return e == hipSuccess ? STPI_OK : hip_fail(e, "warm start");
}

}  // extern "C"
