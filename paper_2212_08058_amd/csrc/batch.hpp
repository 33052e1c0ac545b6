// Batched power iteration over many clips of different length and frame size.
//
// All clips share one filter. Their volumes live in one flat buffer at
// per-clip element offsets. One iteration is one launch of a persistent grid
// (about as many workgroups as fit on the chip at once): each workgroup takes
// tiles from a global work counter until the list is exhausted, so the
// longest clips (listed first) start first and short ones fill the gaps. A
// tile of a clip that has converged is skipped. After the step, one
// workgroup per clip reduces that clip's tile partials and updates its own
// iteration state (scale, residual, stopping), exactly as the single-clip
// chain does. No workgroup ever waits for another, so the grid always drains.
#pragma once

#include <type_traits>

#include "chain.hpp"
#include "forward.hpp"

namespace stpi {

struct ClipDesc {
    int64_t offset;    // element offset of the clip in the flat buffers
    int32_t T, H, W;
    int32_t tile_begin;  // first entry of the clip in the tile list
    int32_t tile_end;
    int32_t pad;
};

struct TileDesc {
    int32_t clip;
    int32_t x0, y0;
    int32_t pad;
};

// Counters shared by the launches of one batched iteration chain.
struct BatchCtl {
    uint32_t next_tile;   // work counter of the running step (reset by the finalisation)
    uint32_t done_clips;  // clips that stopped (converged, capped or failed)
    uint32_t n_active;    // tiles of the clips still iterating (see batch_compact_kernel)
    uint32_t n_clips_active;
};

template <class ST>
struct BatchArgs {
    using CT = typename Compute<ST>::type;
    const ST *f;
    ST *buf0;
    ST *buf1;
    DevState *states;
    const ClipDesc *clips;
    const TileDesc *tiles;
    BatchCtl *ctl;
    double *partials;  // [ntiles][2]
    // clips still iterating, in tile-list order, and the exclusive prefix sums
    // of their tile counts (rebuilt after every step)
    const int32_t *active_clip;
    const int32_t *active_cum;
    int ntiles, nclips;
    int rs;  // the problem's space radius (matrix-core variants)
    Taps<CT> taps;
};

// Wavefronts per SIMD the register allocation must allow: matrix-core tiles
// whose LDS fits twice in a CU's 160 KB are built for two resident workgroups.
template <int TH, int TW, int NTHR, int PIPE, int PAD, int UPLANES>
constexpr int batch_min_waves() {
    if constexpr (PIPE == 3)
        return 2 * (MfmaLds<PIPE, TH, TW, NTHR, PAD, UPLANES>::value * 4 + 1024) <= 160 * 1024 ? 2 * NTHR / 256 : 1;
    else
        return 1;
}

// PIPE: 1 runs each tile through the software-pipelined tile loop, 3 through
// the matrix-core tile loop in product form (see FwdOpP: every clip's
// buffers hold f x g, with g from the clip's own bound on |f|).
template <class ST, int RS, int RT, int TH, int TW, int NTHR, int RY, int QX, int PIPE>
__global__ __launch_bounds__(NTHR, (batch_min_waves<TH, TW, NTHR, PIPE, RS <= 8 ? 8 : 16,
                                                     std::is_same<ST, bf16>::value ? 1 : 2>()))
void batch_step_kernel(BatchArgs<ST> a) {
    using CT = typename Compute<ST>::type;
    using G = Geometry<RS, RT, TH, TW, NTHR, RY, QX>;
    using PG = PipeGeometry<RS, RT, TH, TW, NTHR, RY, QX>;
    constexpr int PAD = RS <= 8 ? 8 : 16;
    static_assert(PIPE != 3 || ((RS == 16 || RS == 8) && sizeof(CT) == 4), "matrix-core batch variants");
    // bfloat16 buffers stage their raw bfloat16 values (one U plane)
    constexpr bool EXACT = PIPE == 3 && std::is_same<ST, bf16>::value;
    __shared__ CT lds[PIPE == 3 ? MfmaLds<PIPE, TH, TW, NTHR, PAD, EXACT ? 1 : 2>::value
                                : (PIPE ? PG::LDS_ELEMS : G::LDS_ELEMS)];
    __shared__ double red[NTHR / 64];
    __shared__ int s_tile;
    __shared__ float tapl[2 * 16 + 1];  // matrix-core variants: space taps centred at 16
    if (a.ctl->done_clips >= (uint32_t)a.nclips) return;
    if constexpr (PIPE == 3) {
        if (threadIdx.x < 2 * 16 + 1) {
            float g = 0.f;
#pragma unroll
            for (int i = 0; i < 2 * RS + 1; ++i) g = (int)threadIdx.x == i + 16 - RS ? (float)a.taps.gs[i] : g;
            tapl[threadIdx.x] = g;
        }
        __syncthreads();
    }
    // Every branch of the tile loop is wave-uniform (readfirstlane values, the
    // wave index), and no branch in it depends on the lane. With the plain
    // form (thread 0 fetches the next tile into LDS, everyone reads it back)
    // the compiler may thread thread 0's "store partials" and "fetch next
    // tile" across the back-edge into a separate path; lanes 1..63 of wave 0
    // then loop back on their own and spin on a tile index that only the
    // parked lane 0 could update. Here wave 0 does the fetch with all lanes
    // active: lane 0 adds one, the others add zero, so the value lane 0 reads
    // back is the claimed tile.
    const int lane = threadIdx.x & 63;
    const int wid = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    for (;;) {
        if (wid == 0) {
            const uint32_t mine = atomicAdd(&a.ctl->next_tile, lane == 0 ? 1u : 0u);
            s_tile = (int)__builtin_amdgcn_readfirstlane(mine);  // all lanes store the same value
        }
        __syncthreads();
        const int g = __builtin_amdgcn_readfirstlane(s_tile);
        __syncthreads();
        if (g >= (int)__builtin_amdgcn_readfirstlane(a.ctl->n_active)) break;
        // the active clip holding claimed tile g: last i with active_cum[i] <= g
        int lo = 0, hi = __builtin_amdgcn_readfirstlane(a.ctl->n_clips_active) - 1;
        while (lo < hi) {
            const int mid = (lo + hi + 1) >> 1;
            if (__builtin_amdgcn_readfirstlane(a.active_cum[mid]) <= g) lo = mid;
            else hi = mid - 1;
        }
        const int aclip = __builtin_amdgcn_readfirstlane(a.active_clip[lo]);
        const int t = __builtin_amdgcn_readfirstlane(a.clips[aclip].tile_begin) + g -
                      __builtin_amdgcn_readfirstlane(a.active_cum[lo]);
        const int clip = __builtin_amdgcn_readfirstlane(a.tiles[t].clip);
        const int tx0 = __builtin_amdgcn_readfirstlane(a.tiles[t].x0);
        const int ty0 = __builtin_amdgcn_readfirstlane(a.tiles[t].y0);
        const ClipDesc cd = a.clips[clip];
        const DevState *st_ = a.states + clip;
        double d1 = 0.0, d2 = 0.0;
        if (!__builtin_amdgcn_readfirstlane(st_->done)) {
            const int cur = __builtin_amdgcn_readfirstlane(st_->cur);
            FwdOp<ST> op;
            op.f = a.f + cd.offset;
            op.src = (cur ? a.buf1 : a.buf0) + cd.offset;
            op.dst = (cur ? a.buf0 : a.buf1) + cd.offset;
            op.vout = nullptr;
            op.scale = (CT)st_->scale;
            op.plane = (size_t)cd.H * cd.W;
            op.pbytes = (uint32_t)(op.plane * sizeof(ST));
            const int T = __builtin_amdgcn_readfirstlane(cd.T);
            const int H = __builtin_amdgcn_readfirstlane(cd.H), W = __builtin_amdgcn_readfirstlane(cd.W);
            op.cut = tx0 + TW > W;  // 4-wide epilogue loads read past the right edge here
            if constexpr (PIPE == 3) {
                // the single-clip product-form step's arithmetic, on this clip's state
                const float fb = __uint_as_float(st_->ubound);
                const int e = bound_exponent(fb, PRODUCT_ELIM);
                const bool first = __builtin_amdgcn_readfirstlane(st_->pform) == 2;
                FwdOpP<ST> pp;
                pp.f = op.f;
                pp.src = first ? op.f : op.src;
                pp.dst = op.dst;
                pp.gout = ldexpf(1.f, -2 * e);
                pp.ginv_out = ldexp(1.0, 2 * e);
                pp.ginv_in = first ? 1.0 : pp.ginv_out;
                pp.plane = op.plane;
                pp.pbytes = op.pbytes;
                pp.cut = tx0 + TW > W;
                // staging power of two from the input's own maximum (as the single-clip step)
                const float win = first ? fb : __uint_as_float(st_->wmax[cur]);
                float umul;
                if constexpr (EXACT) {
                    const int ein = bound_exponent((float)((double)win * pp.ginv_in), 100);
                    pp.sg = (float)(st_->scale * ldexp(1.0, ein - 10 - 2 * e));
                    umul = (float)ldexp(pp.ginv_in, 10 - ein);
                } else {
                    const int ein = bound_exponent((float)((double)win * st_->scale * pp.ginv_in), 100);
                    pp.sg = ldexpf(1.f, ein - 10 - 2 * e);
                    umul = (float)(st_->scale * ldexp(1.0, 10 - ein) * pp.ginv_in);
                }
                stencil_tile_mfma<CT, RT, TH, TW, NTHR, PAD, EXACT>(pp, a.taps, tapl, umul, a.rs, T, 0, T, H, W, tx0,
                                                              ty0, lds, d1, d2);
                d1 *= pp.ginv_in * pp.ginv_out;
                d2 *= pp.ginv_out * pp.ginv_out;
                const float m = block_max<NTHR>(pp.wmax, reinterpret_cast<float *>(red));
                if (threadIdx.x == 0 && m > 0.f) atomicMax(&a.states[clip].wmax[cur ^ 1], __float_as_uint(m));
            } else if constexpr (PIPE)
                stencil_tile_pipe<CT, RS, RT, TH, TW, NTHR, RY, QX>(op, a.taps, T, 0, T, H, W, tx0, ty0, lds, d1, d2);
            else
                stencil_tile<CT, RS, RT, TH, TW, NTHR, RY, QX>(op, a.taps, T, 0, T, H, W, tx0, ty0, lds, d1, d2);
            // the next tile's staging reuses the LDS tiles
            __syncthreads();
        }
        // block sums land in thread 0 (lane 0 of wave 0); wave 0 broadcasts and stores them
        const double s1 = block_sum<NTHR>(d1, red);
        const double s2 = block_sum<NTHR>(d2, red);
        if (wid == 0) {
            const double b1 = __shfl(s1, 0, 64), b2 = __shfl(s2, 0, 64);
            a.partials[2 * (size_t)t] = b1;  // same address and value in every lane
            a.partials[2 * (size_t)t + 1] = b2;
        }
    }
}

// One workgroup per clip: the clip's step finalisation (see finalize_kernel).
// With the rise check (a warm start), a clip whose second residual exceeds
// its first restarts from the uniform start 1/sqrt(n) on the device: its
// iteration count keeps the two discarded steps.
__device__ __forceinline__ void finalize_state(DevState *s, double p1, double p2, BatchCtl *ctl, double n) {
    const double scale = s->scale;
    const double nz = sqrt(p2);
    bool stop = false;
    if (!isfinite(nz) || !isfinite(p1)) {
        s->flags |= FLAG_NONFINITE;
        stop = true;
    } else if (nz == 0.0) {
        s->flags |= FLAG_ZERO;
        stop = true;
    } else {
        const double c = scale * p1 / nz;
        s->rayleigh = scale * p1;
        s->lambda = nz;
        s->residual = sqrt(fmax(0.0, 2.0 - 2.0 * c));
        s->scale = 1.0 / nz;
        s->wmax[s->cur] = 0u;  // the buffer just read is the next step's output
        s->cur ^= 1;
        s->iters += 1;
        if (s->pform == 2) s->pform = 1;
        s->refill = 0;
        if (s->iters <= 2) s->first_res[s->iters - 1] = s->residual;
        if (s->check_rise && s->iters == 2 && !(s->first_res[1] <= s->first_res[0])) {
            s->flags |= FLAG_ROSE;
            s->check_rise = 0;
            s->scale = 1.0 / sqrt(n);
            s->wmax[0] = s->wmax[1] = 0u;
            if (s->pform) s->pform = 2;  // product form: the next step stages f itself
            else s->refill = 1;          // plain form: batch_refill_kernel writes the constant 1
        } else if (s->tol > 0.0 && s->residual < s->tol) {
            s->converged = 1;
            stop = true;
        }
        if (s->iters >= s->max_iters) stop = true;
    }
    if (stop) {
        s->done = 1;
        atomicAdd(&ctl->done_clips, 1u);
    }
}

}  // namespace stpi

namespace stpi {

// Per-storage-type pieces of the batched chain (instantiated in kernels_<type>.hip).

struct BatchLaunch {
    const void *f;
    void *buf0, *buf1;
    DevState *states;
    const ClipDesc *clips;
    const TileDesc *tiles;
    BatchCtl *ctl;
    double *partials;
    const int32_t *active_clip, *active_cum;
    int ntiles, nclips, grid;
    double gs[2 * 16 + 1];
    double gt[2 * 8 + 1];
};

struct BatchVariant {
    int RS, RT, TH, TW, NTHR, RY, QX, PIPE;
    hipError_t (*launch)(const BatchLaunch &, hipStream_t);
    int (*blocks_per_cu)();
};

template <class ST, int RS, int RT, int TH, int TW, int NTHR, int RY, int QX, int PIPE>
hipError_t launch_batch(const BatchLaunch &L, hipStream_t stream) {
    using CT = typename Compute<ST>::type;
    BatchArgs<ST> a;
    a.f = (const ST *)L.f;
    a.buf0 = (ST *)L.buf0;
    a.buf1 = (ST *)L.buf1;
    a.states = L.states;
    a.clips = L.clips;
    a.tiles = L.tiles;
    a.ctl = L.ctl;
    a.partials = L.partials;
    a.active_clip = L.active_clip;
    a.active_cum = L.active_cum;
    a.ntiles = L.ntiles;
    a.nclips = L.nclips;
    a.rs = 0;
    for (int d = 1; d <= 16; ++d)
        if (L.gs[16 + d] != 0.0) a.rs = d;
    for (int i = 0; i < 2 * 16 + 1; ++i) a.taps.gs[i] = CT(0);
    for (int i = 0; i < 2 * 8 + 1; ++i) a.taps.gt[i] = CT(0);
    for (int d = -RS; d <= RS; ++d) a.taps.gs[d + RS] = (CT)L.gs[d + 16];
    for (int d = -RT; d <= RT; ++d) a.taps.gt[d + RT] = (CT)L.gt[d + 8];
    hipLaunchKernelGGL((batch_step_kernel<ST, RS, RT, TH, TW, NTHR, RY, QX, PIPE>), dim3(L.grid), dim3(NTHR), 0,
                       stream, a);
    return hipGetLastError();
}

template <class ST, int RS, int RT, int TH, int TW, int NTHR, int RY, int QX, int PIPE>
int batch_blocks_per_cu() {
    int n = 0;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&n, batch_step_kernel<ST, RS, RT, TH, TW, NTHR, RY, QX, PIPE>,
                                                     NTHR, 0) != hipSuccess)
        n = 1;
    return n > 0 ? n : 1;
}

constexpr int BATCH_NORM_BLOCKS = 64;  // workgroups per clip in the per-clip reductions

// Plain-form batch after a rejected warm start: the current buffer of every
// clip marked for it <- 1 (the finalisation already set the uniform scale).
template <class ST>
__global__ void batch_refill_kernel(ST *buf0, ST *buf1, const ClipDesc *clips, const DevState *states) {
    using CT = typename Compute<ST>::type;
    const DevState *s = states + blockIdx.y;
    if (!s->refill) return;
    const ClipDesc cd = clips[blockIdx.y];
    ST *x = (s->cur ? buf1 : buf0) + cd.offset;
    const size_t n = (size_t)cd.T * cd.H * cd.W;
    for (size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (size_t)gridDim.x * blockDim.x)
        st(x + i, CT(1));
}

// x[clip] <- 1 (uniform start, scale set by the init kernel)
template <class ST>
__global__ void batch_fill_ones_kernel(ST *x, const ClipDesc *clips) {
    using CT = typename Compute<ST>::type;
    const ClipDesc cd = clips[blockIdx.y];
    const size_t n = (size_t)cd.T * cd.H * cd.W;
    for (size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (size_t)gridDim.x * blockDim.x)
        st(x + cd.offset + i, CT(1));
}

// partials[(clip * BATCH_NORM_BLOCKS + b) * 2] = sum of squares of the clip's x
template <class ST>
__global__ void batch_sumsq_kernel(const ST *x, const ClipDesc *clips, double *partials) {
    __shared__ double red[256 / 64];
    const ClipDesc cd = clips[blockIdx.y];
    const size_t n = (size_t)cd.T * cd.H * cd.W;
    double a = 0.0;
    for (size_t i = (size_t)blockIdx.x * 256 + threadIdx.x; i < n; i += (size_t)gridDim.x * 256) {
        const double v = (double)ld(x + cd.offset + i);
        a += v * v;
    }
    const double s = block_sum<256>(a, red);
    if (threadIdx.x == 0) {
        partials[2 * ((size_t)blockIdx.y * BATCH_NORM_BLOCKS + blockIdx.x)] = s;
        partials[2 * ((size_t)blockIdx.y * BATCH_NORM_BLOCKS + blockIdx.x) + 1] = 0.0;
    }
}

// states[clip].ubound = max |f| over the clip (float bits: non-negative
// floats order as their bit patterns), for the matrix-core variants.
template <class ST>
__global__ void batch_bound_kernel(const ST *f, const ClipDesc *clips, DevState *states) {
    __shared__ float red[256 / 64];
    const ClipDesc cd = clips[blockIdx.y];
    const size_t n = (size_t)cd.T * cd.H * cd.W;
    float m = 0.f;
    for (size_t i = (size_t)blockIdx.x * 256 + threadIdx.x; i < n; i += (size_t)gridDim.x * 256)
        m = fmaxf(m, fabsf((float)ld(f + cd.offset + i)));
#pragma unroll
    for (int off = 32; off >= 1; off >>= 1) m = fmaxf(m, __shfl_xor(m, off, 64));
    if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = m;
    __syncthreads();
    if (threadIdx.x == 0) {
        for (int i = 1; i < 256 / 64; ++i) m = fmaxf(m, red[i]);
        atomicMax(&states[blockIdx.y].ubound, __float_as_uint(m));
    }
}

// Product-form start from the caller's x, per clip: buffer 1 <- f x g.
template <class ST>
__global__ void batch_to_product_kernel(const ST *f, const ST *x, ST *w, const ClipDesc *clips, DevState *states) {
    using CT = typename Compute<ST>::type;
    __shared__ float red[256 / 64];
    const ClipDesc cd = clips[blockIdx.y];
    DevState *s = states + blockIdx.y;
    const CT g = (CT)ldexp(1.0, -2 * bound_exponent(__uint_as_float(s->ubound), PRODUCT_ELIM));
    const size_t n = (size_t)cd.T * cd.H * cd.W;
    float m = 0.f;
    for (size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (size_t)gridDim.x * blockDim.x) {
        const CT v = (ld(f + cd.offset + i) * ld(x + cd.offset + i)) * g;
        st(w + cd.offset + i, v);
        m = fmaxf(m, fabsf((float)stored_value(w + cd.offset + i, v)));
    }
    m = block_max<256>(m, red);
    if (threadIdx.x == 0 && m > 0.f) atomicMax(&s->wmax[1], __float_as_uint(m));
    if (blockIdx.x == 0 && threadIdx.x == 0) {
        s->cur = 1;
        s->pform = 1;
    }
}

// Final pass of a product-form batch, per clip (as from_product_kernel).
template <class ST>
__global__ void batch_from_product_kernel(ST *x, const ST *buf1, const ST *f, const ClipDesc *clips,
                                          const DevState *states) {
    using CT = typename Compute<ST>::type;
    const ClipDesc cd = clips[blockIdx.y];
    const DevState *s = states + blockIdx.y;
    const size_t n = (size_t)cd.T * cd.H * cd.W;
    const size_t i0 = (size_t)blockIdx.x * blockDim.x + threadIdx.x, stride = (size_t)gridDim.x * blockDim.x;
    if (s->pform == 2) {
        const CT c = (CT)s->scale;
        for (size_t i = i0; i < n; i += stride) st(x + cd.offset + i, c);
        return;
    }
    const ST *src = (s->cur ? buf1 : x) + cd.offset;
    const double m = s->scale * ldexp(1.0, 2 * bound_exponent(__uint_as_float(s->ubound), PRODUCT_ELIM));
    for (size_t i = i0; i < n; i += stride) {
        const CT fv = ld(f + cd.offset + i);
        st(x + cd.offset + i, fv != CT(0) ? (CT)((double)ld(src + i) / (double)fv * m) : CT(0));
    }
}

// x[clip] <- scale_clip * (current iterate of the clip)
template <class ST>
__global__ void batch_normalize_kernel(ST *x, const ST *buf1, const ClipDesc *clips, const DevState *states) {
    using CT = typename Compute<ST>::type;
    const ClipDesc cd = clips[blockIdx.y];
    const DevState *s = states + blockIdx.y;
    const ST *src = (s->cur ? buf1 : x) + cd.offset;
    const CT scale = (CT)s->scale;
    const size_t n = (size_t)cd.T * cd.H * cd.W;
    for (size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (size_t)gridDim.x * blockDim.x)
        st(x + cd.offset + i, scale * ld(src + i));
}

}  // namespace stpi
