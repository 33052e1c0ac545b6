// Matrix-core form of the step's two spatial passes (space radius up to 16).
//
// A 1D Gaussian pass over a tile is a product with a banded Toeplitz matrix,
// so both spatial passes of the separable filter (the 1D passes of Sec. 4, "Computational complexity",
// along y then x) run as v_mfma_f32_16x16x32_f16 products. To keep
// float accuracy, every operand is split into two half-precision parts,
// a = a_hi + a_lo with a_hi = fp16(a) and a_lo = fp16(a - a_hi) (about 22
// significant bits), and each product is formed from the three terms that
// matter: hi*hi + hi*lo + lo*hi (the dropped lo*lo term and the split
// residuals are below 2^-21 of each product). Products accumulate in float.
//
// Range. The staged input is u' = f x_stored scale 2^S, where scale makes the
// iterate unit and 2^S is chosen on the device from a bound B >= |f x scale|
// so that |u'| < 2^10; the y-pass output is then below (2 PAD + 1) 2^10 <= 33 *
// 2^10 (the taps are <= 1), inside half precision. The output picks up 2^-S in
// the epilogue's scale, so z is the same as in the plain form. B is the
// actual maximum (single step: max |f x| |scale|; iteration chains: max |w|
// of the stored iterate, collected by the step that wrote it), so the
// largest staged value lies in [2^9, 2^10) and the split keeps about 22
// significant bits for every value within 2^14 of it; smaller values keep an
// absolute error below 2^-24, i.e. 2^-33 of the largest.
//
// Tile. A workgroup owns TH x TW outputs (multiples of 16) and streams its
// frames as the plain tile loop does (three-stage pipeline, one barrier per
// phase, the same t-ring and epilogue). Each phase issues the epilogue's
// loads, then the matrix-core products of both passes (they read buffers
// written before the phase's barrier), then does the vector work (staging,
// t-ring, epilogue) while those run, and stores the y-pass result last.
// Per frame:
//   stage:  u' on the (TH + 2 PAD) x (TW + 2 PAD) slab around the tile (PAD =
//           8 or 16, at least the space radius), split into
//           hi and lo planes stored column-major (U^T[c][k], k = slab row),
//           each thread writing 8 consecutive rows of one column (16 bytes);
//   y-pass: for each 16 x 16 block of Y (16 tile rows x 16 slab columns),
//           Y^T = sum_kb U^T[cols][32 kb .. 32 kb + 32) * Bband_kb (KB = 2
//           K blocks of 32 for PAD = 16, one for PAD = 8), giving
//           each lane 4 consecutive columns of one row, stored row-major in
//           hi and lo planes;
//   x-pass: for each 16 x 16 output block, Out^T = sum_kb Bband_kb^T *
//           Y^T[32 kb ..], again 4 consecutive columns of one row per lane,
//           which feed the t-ring (2 RT + 1 register slots) and the epilogue.
// Both band matrices hold g(32 kb + k - PAD - i) at (row i, col k) in the
// operand layout, so one set of tap registers serves as the y-pass B operand
// and the x-pass A operand (bfloat16 inputs stage their raw values and take
// a second, bfloat16 set for the y-pass: stencil_tile_mfma's EXACT). Rows and columns of the slab beyond the space
// radius are staged as zeros; with PAD = 16 the 16 extra U rows and Y columns
// that the last K block of the bottom / right blocks reads are zeroed once.
#pragma once

#include "stencil.hpp"

namespace stpi {

typedef _Float16 half8_t __attribute__((ext_vector_type(8)));
typedef __bf16 bf16x8_t __attribute__((ext_vector_type(8)));
typedef unsigned short u16x8_t __attribute__((ext_vector_type(8)));
typedef _Float16 half4_t __attribute__((ext_vector_type(4)));
typedef float float4_t __attribute__((ext_vector_type(4)));

// Halves per LDS line: a multiple of 8 (16-byte rows) with an odd number of
// 16-byte chunks, so 16-byte accesses of lanes one line apart spread over
// the banks.
constexpr int mfma_pitch(int n) {
    const int p = (n + 7) & ~7;
    return ((p / 8) % 2 == 1) ? p : p + 8;
}

// PAD (8 or 16) is the slab margin, at least the space radius. An output
// block of 16 rows (columns) reads 16 + 2 PAD slab rows (columns), that is KB
// K blocks of 32 (the last 16 of them zero weight when PAD = 16).
// UPLANES: 16-bit planes per staged U buffer: 2 (half-precision hi and lo)
// in general, 1 for bfloat16 inputs staged as they are (see
// stencil_tile_mfma's EXACT).
template <int TH, int TW, int NTHR, int PAD, int UPLANES = 2>
struct MfmaGeometry {
    static constexpr int KB = (16 + 2 * PAD + 31) / 32;
    static constexpr int MB = TH / 16, NB = TW / 16;  // output blocks down / across
    static constexpr int SR = TH + 2 * PAD, SC = TW + 2 * PAD;  // staged slab rows / columns
    static constexpr int UK = TH - 16 + 32 * KB;      // U^T column length read by the y-pass
    static constexpr int UP = mfma_pitch(UK);
    static constexpr int YW = TW - 16 + 32 * KB;      // Y row length read by the x-pass
    static constexpr int YP = mfma_pitch(YW);
    static constexpr int UPL = SC * UP;               // halves per U plane
    static constexpr int YPL = TH * YP;               // halves per Y plane
    static constexpr int UBUF = UPLANES * UPL;        // hi (and lo) planes
    static constexpr int YBUF = 2 * YPL;
    static constexpr int LDS_HALVES = 2 * UBUF + 2 * YBUF;  // double-buffered
    static constexpr int LDS_FLOATS = LDS_HALVES / 2;
    static constexpr int NG = SR / 8;                 // 8-row groups per slab column
    static constexpr int NITEM = SC * NG;             // staging items
    static constexpr int IPS = (NITEM + NTHR - 1) / NTHR;
    static constexpr int NPF = 8 * IPS;               // prefetched elements per thread
    static constexpr int NWAVE = NTHR / 64;
    static constexpr int NYC = SC / 16;               // y-pass block columns
    static constexpr int NYB = MB * NYC;              // y-pass blocks
    static constexpr int NXB = MB * NB;               // x-pass blocks
    static constexpr int YPW = (NYB + NWAVE - 1) / NWAVE;
    static constexpr int XPW = NXB / NWAVE;           // x-pass blocks per wavefront
    static_assert(TH % 16 == 0 && TW % 16 == 0, "tile of whole 16 x 16 blocks");
    static_assert(PAD == 8 || PAD == 16, "slab margin 8 or 16");
    static_assert(NXB % NWAVE == 0, "x-pass blocks must split evenly over the wavefronts");
    static_assert(NB % XPW == 0, "a wavefront's x-pass blocks lie in one block row");
    static_assert(LDS_HALVES % 2 == 0 && LDS_HALVES * 2 <= 160 * 1024, "LDS");
};

// LDS floats of a tile loop kind (instantiates the geometry only for PIPE 3).
template <int PIPE, int TH, int TW, int NTHR, int PAD, int UPLANES = 2>
struct MfmaLds {
    static constexpr int value = 1;
};
template <int TH, int TW, int NTHR, int PAD, int UPLANES>
struct MfmaLds<3, TH, TW, NTHR, PAD, UPLANES> {
    static constexpr int value = MfmaGeometry<TH, TW, NTHR, PAD, UPLANES>::LDS_FLOATS;
};

// Staging item m of thread tid. When the items do not fill the last round,
// that round goes to the highest threads: the y-pass's extra blocks go to the
// lowest wavefronts, so no wavefront carries both.
template <class G, int NTHR>
__device__ __forceinline__ int stage_item(int tid, int m) {
    if (G::NITEM % NTHR != 0 && m == G::IPS - 1) return (G::IPS - 1) * NTHR + (NTHR - 1 - tid);
    return tid + m * NTHR;
}

__device__ __forceinline__ void split_half(float v, _Float16 &hi, _Float16 &lo) {
    hi = (_Float16)v;
    lo = (_Float16)(v - (float)hi);
}

// Launders a constant so the compiler keeps it as an operand (fma(x, 1, y)
// would otherwise fold to an add, which has no mixed-precision form).
__device__ __forceinline__ float opaque(float v) {
    asm volatile("" : "+v"(v));
    return v;
}

// Splits 4 floats into half-precision hi and lo parts: hi = fp16(v),
// lo = fp16(v - hi) (one mixed-precision fma per element).
__device__ __forceinline__ void split4(const float4_t &v, half4_t &h, half4_t &l, float one) {
#pragma unroll
    for (int j = 0; j < 4; ++j) h[j] = (_Float16)v[j];
#pragma unroll
    for (int j = 0; j < 4; ++j) l[j] = (_Float16)__builtin_fmaf(-(float)h[j], one, v[j]);
}

// y-pass products of one 16 x 16 block of Y (one dependency chain).
template <class G>
__device__ __forceinline__ float4_t mfma_yblock_mma(const _Float16 *U, int b, int lane, const half8_t (&thi)[G::KB],
                                                    const half8_t (&tlo)[G::KB]) {
    const int rb = b / G::NYC, cb = b % G::NYC;
    const int li = lane & 15, lg = lane >> 4;
    const _Float16 *p = U + (16 * cb + li) * G::UP + 16 * rb + 8 * lg;
    float4_t acc = {0.f, 0.f, 0.f, 0.f};
#pragma unroll
    for (int kb = 0; kb < G::KB; ++kb) {
        const half8_t ah = *reinterpret_cast<const half8_t *>(p + 32 * kb);
        const half8_t al = *reinterpret_cast<const half8_t *>(p + G::UPL + 32 * kb);
        acc = __builtin_amdgcn_mfma_f32_16x16x32_f16(ah, thi[kb], acc, 0, 0, 0);
        acc = __builtin_amdgcn_mfma_f32_16x16x32_f16(ah, tlo[kb], acc, 0, 0, 0);
        acc = __builtin_amdgcn_mfma_f32_16x16x32_f16(al, thi[kb], acc, 0, 0, 0);
    }
    return acc;
}

// The same for bfloat16 inputs staged as they are (one plane of raw
// bfloat16): bfloat16 products with the taps (times the staging multiplier)
// split into two bfloat16 parts, hi + lo (about 16 significant bits).
template <class G>
__device__ __forceinline__ float4_t mfma_yblock_mma_bf16(const _Float16 *U, int b, int lane,
                                                         const bf16x8_t (&bhi)[G::KB], const bf16x8_t (&blo)[G::KB]) {
    const int rb = b / G::NYC, cb = b % G::NYC;
    const int li = lane & 15, lg = lane >> 4;
    const _Float16 *p = U + (16 * cb + li) * G::UP + 16 * rb + 8 * lg;
    float4_t acc = {0.f, 0.f, 0.f, 0.f};
#pragma unroll
    for (int kb = 0; kb < G::KB; ++kb) {
        const bf16x8_t a = *reinterpret_cast<const bf16x8_t *>(p + 32 * kb);
        acc = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a, bhi[kb], acc, 0, 0, 0);
        acc = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a, blo[kb], acc, 0, 0, 0);
    }
    return acc;
}

// Stores a y-pass block: split into the Y hi and lo planes.
template <class G>
__device__ __forceinline__ void mfma_yblock_store(_Float16 *Y, int b, int lane, const float4_t &acc, float one) {
    const int rb = b / G::NYC, cb = b % G::NYC;
    const int li = lane & 15, lg = lane >> 4;
    half4_t h, l;
    split4(acc, h, l, one);
    _Float16 *q = Y + (16 * rb + li) * G::YP + 16 * cb + 4 * lg;
    *reinterpret_cast<half4_t *>(q) = h;
    *reinterpret_cast<half4_t *>(q + G::YPL) = l;
}

// x-pass products of one 16 x 16 output block (one dependency chain).
template <class G>
__device__ __forceinline__ float4_t mfma_xblock_mma(const _Float16 *Y, int b, int lane, const half8_t (&thi)[G::KB],
                                                    const half8_t (&tlo)[G::KB]) {
    const int rb = b / G::NB, ob = b % G::NB;
    const int li = lane & 15, lg = lane >> 4;
    const _Float16 *p = Y + (16 * rb + li) * G::YP + 16 * ob + 8 * lg;
    float4_t acc = {0.f, 0.f, 0.f, 0.f};
#pragma unroll
    for (int kb = 0; kb < G::KB; ++kb) {
        const half8_t bh = *reinterpret_cast<const half8_t *>(p + 32 * kb);
        const half8_t bl = *reinterpret_cast<const half8_t *>(p + G::YPL + 32 * kb);
        acc = __builtin_amdgcn_mfma_f32_16x16x32_f16(thi[kb], bh, acc, 0, 0, 0);
        acc = __builtin_amdgcn_mfma_f32_16x16x32_f16(tlo[kb], bh, acc, 0, 0, 0);
        acc = __builtin_amdgcn_mfma_f32_16x16x32_f16(thi[kb], bl, acc, 0, 0, 0);
    }
    return acc;
}

// Streams one tile through frames [t0, t1) (reading [t0 - RT, t1 + RT) clipped
// to the clip). Op is the forward step's FwdOp; umul = scale * 2^S multiplies
// f * x at staging and op.scale must be 2^-S. rs is the problem's space
// radius (slab rows and columns beyond it are not read). lds holds
// MfmaGeometry::LDS_FLOATS floats; tapl holds the 33 space taps centred at 16.
// EXACT: the inputs are bfloat16 values (op.input returns them exactly as
// floats) and umul is a power of two: U holds the inputs as they are, one
// plane of raw bfloat16 with no conversion at staging, and the y-pass takes
// umul into its taps (bfloat16 products, mfma_yblock_mma_bf16). The result
// is stored in bfloat16, so taps with about 16 significant bits suffice.
template <class CT, int RT, int TH, int TW, int NTHR, int PAD, bool EXACT = false, class Op>
__device__ __forceinline__ void stencil_tile_mfma(const Op &op, const Taps<CT> &tp, const float *tapl, float umul,
                                                  int rs, int T, int t0, int t1, int H, int W, int x0, int y0,
                                                  float *lds, double &d1, double &d2) {
    using G = MfmaGeometry<TH, TW, NTHR, PAD, EXACT ? 1 : 2>;
    constexpr int NPF = G::NPF, IPS = G::IPS, NTS = 2 * RT + 1, XPW = G::XPW;
    constexpr uint32_t ESZ = Op::ESZ;
    const int tid = threadIdx.x;
    const int lane = tid & 63;
    const int wid = __builtin_amdgcn_readfirstlane(tid >> 6);
    _Float16 *const U0 = reinterpret_cast<_Float16 *>(lds);
    _Float16 *const Y0 = U0 + 2 * G::UBUF;

    // band taps in the operand layout: lane l, element j of K block kb holds
    // g(32 kb + 8 (l / 16) + j - PAD - l % 16)
    half8_t thi[G::KB], tlo[G::KB];
#pragma unroll
    for (int kb = 0; kb < G::KB; ++kb)
#pragma unroll
        for (int j = 0; j < 8; ++j) {
            const int d = 32 * kb + 8 * (lane >> 4) + j - PAD - (lane & 15);
            const float g = (d >= -16 && d <= 16) ? tapl[d + 16] : 0.f;
            _Float16 h, l;
            split_half(g, h, l);
            thi[kb][j] = h;
            tlo[kb][j] = l;
        }
    // EXACT: the y-pass taps times umul (a power of two, so exact in float) as
    // two bfloat16 parts
    bf16x8_t bhi[G::KB], blo[G::KB];
    if constexpr (EXACT) {
#pragma unroll
        for (int kb = 0; kb < G::KB; ++kb)
#pragma unroll
            for (int j = 0; j < 8; ++j) {
                const int d = 32 * kb + 8 * (lane >> 4) + j - PAD - (lane & 15);
                const float g = ((d >= -16 && d <= 16) ? tapl[d + 16] : 0.f) * umul;
                const __bf16 h = (__bf16)g;
                bhi[kb][j] = h;
                blo[kb][j] = (__bf16)(g - (float)h);
            }
    }

    // zero the U^T rows [SR, UK) and the Y columns [SC, YW) of both buffers
    // (none when PAD = 8)
    for (int i = tid; i < 2 * (EXACT ? 1 : 2) * G::SC * (G::UK - G::SR); i += NTHR) {
        const int k = i % (G::UK - G::SR), rest = i / (G::UK - G::SR);
        const int c = rest % G::SC, plane = rest / G::SC;  // plane: buffer * planes + hi/lo
        U0[plane * G::UPL + c * G::UP + G::SR + k] = (_Float16)0.f;
    }
    for (int i = tid; i < 2 * 2 * TH * (G::YW - G::SC); i += NTHR) {
        const int k = i % (G::YW - G::SC), rest = i / (G::YW - G::SC);
        const int r = rest % TH, plane = rest / TH;
        Y0[plane * G::YPL + r * G::YP + G::SC + k] = (_Float16)0.f;
    }

    // staging offsets: item m of this thread is slab column c, rows 8 g .. 8 g + 7
    uint32_t poff[NPF];
#pragma unroll
    for (int m = 0; m < IPS; ++m) {
        const int it = stage_item<G, NTHR>(tid, m);
        const int c = it % G::SC, g = it / G::SC;
        const int gx = x0 - PAD + c;
        const bool colok = it < G::NITEM && c >= PAD - rs && c < TW + PAD + rs && (unsigned)gx < (unsigned)W;
#pragma unroll
        for (int j = 0; j < 8; ++j) {
            const int r = 8 * g + j;
            const int gy = y0 - PAD + r;
            const bool ok = colok && r >= PAD - rs && r < TH + PAD + rs && (unsigned)gy < (unsigned)H;
            poff[8 * m + j] = ok ? (uint32_t)(gy * W + gx) * ESZ : OOB;
        }
    }
    // output offsets: x-pass block i of this wavefront, row li, columns 4 lg .. 4 lg + 3.
    // The epilogue's operands move in 4-wide loads at the first offset of each
    // group: op.cut must be set where the tile reaches past the right edge.
    uint32_t ooff[XPW][4];
#pragma unroll
    for (int i = 0; i < XPW; ++i) {
        const int b = wid * XPW + i;
        const int rb = b / G::NB, ob = b % G::NB;
        const int gy = y0 + 16 * rb + (lane & 15);
#pragma unroll
        for (int q = 0; q < 4; ++q) {
            const int gx = x0 + 16 * ob + 4 * (lane >> 4) + q;
            ooff[i][q] = (gy < H && gx < W) ? (uint32_t)(gy * W + gx) * ESZ : OOB;
        }
    }

    CT acc[NTS][XPW][4];
#pragma unroll
    for (int s = 0; s < NTS; ++s)
#pragma unroll
        for (int i = 0; i < XPW; ++i)
#pragma unroll
            for (int q = 0; q < 4; ++q) acc[s][i][q] = CT(0);

    const FrameWalk<RT> fw(T, t0, t1);  // frame order (the last segment walks backward)
    const int nin = fw.nin;
    typename Op::template Raw<NPF> pf;
    op.template fetch<NPF>(fw.in(0), poff, pf);
    typename Op::template OutRaw<XPW, 4> oraw;

    const int nphase = fw.nstep + 2;
    const float one = opaque(1.f);
    ring_loop<NTS, -2>(nphase, [&](auto ring_pos, int p) __attribute__((always_inline)) {
        constexpr int J = decltype(ring_pos)::value;
        const int tx = p - 2;
        const int tout = fw.out(tx);
        const bool emit = tx >= 0 && tout >= t0 && tout < t1;
        const bool xlive = tx >= 0 && tx < nin;
        const bool ylive = p >= 1 && p - 1 < nin;
        // the epilogue's loads go first: they have the whole phase to arrive.
        // Both load groups are issued in every phase (on an empty range when
        // not needed) so that the memory-counter waits before each use allow
        // for the younger group instead of draining it.
        op.template fetch_out<XPW, 4>(tout, ooff, oraw, emit);
        // matrix-core products of both passes (frames p - 2 and p - 1; the
        // buffers they read were written before the last barrier), issued
        // before the vector work of the phase so that they run beside it
        float4_t xa[XPW];
        if (xlive) {
            const _Float16 *Y = Y0 + (tx & 1) * G::YBUF;
#pragma unroll
            for (int i = 0; i < XPW; ++i) xa[i] = mfma_xblock_mma<G>(Y, wid * XPW + i, lane, thi, tlo);
        }
        float4_t ya[G::YPW];
        if (ylive) {
            const _Float16 *U = U0 + ((p - 1) & 1) * G::UBUF;
#pragma unroll
            for (int m = 0; m < G::YPW; ++m) {
                const int b = wid + m * G::NWAVE;
                if (G::NYB % G::NWAVE == 0 || b < G::NYB) {
                    if constexpr (EXACT)
                        ya[m] = mfma_yblock_mma_bf16<G>(U, b, lane, bhi, blo);
                    else
                        ya[m] = mfma_yblock_mma<G>(U, b, lane, thi, tlo);
                }
            }
        }
        if (p < nin) {
            _Float16 *U = U0 + (p & 1) * G::UBUF;
#pragma unroll
            for (int m = 0; m < IPS; ++m) {
                const int it = stage_item<G, NTHR>(tid, m);
                if (G::NITEM % NTHR == 0 || m < IPS - 1 || it < G::NITEM) {
                    const int c = it % G::SC, g = it / G::SC;
                    _Float16 *q = U + c * G::UP + 8 * g;
                    if constexpr (EXACT) {
                        u16x8_t h;  // the inputs' own bfloat16 bits
#pragma unroll
                        for (int j = 0; j < 8; ++j)
                            h[j] = (unsigned short)(__float_as_uint(op.template input<NPF>(pf, 8 * m + j)) >> 16);
                        *reinterpret_cast<u16x8_t *>(q) = h;
                    } else {
                        half8_t h, l;
#pragma unroll
                        for (int j = 0; j < 8; ++j) {
                            _Float16 a, b;
                            split_half(op.template input<NPF>(pf, 8 * m + j) * umul, a, b);
                            h[j] = a;
                            l[j] = b;
                        }
                        *reinterpret_cast<half8_t *>(q) = h;
                        *reinterpret_cast<half8_t *>(q + G::UPL) = l;
                    }
                }
            }
        }
        op.template fetch<NPF>(fw.in(p + 1), poff, pf, p + 1 < nin);
        if (tx >= 0) {
            CT v[XPW][4];
#pragma unroll
            for (int i = 0; i < XPW; ++i)
#pragma unroll
                for (int q = 0; q < 4; ++q) v[i][q] = xlive ? xa[i][q] : CT(0);
            ring_step<J, CT, RT, XPW, 4>(acc, v, tp, xlive, emit, tout, op, ooff, oraw, d1, d2);
        }
        if (ylive) {
            _Float16 *Y = Y0 + ((p - 1) & 1) * G::YBUF;
#pragma unroll
            for (int m = 0; m < G::YPW; ++m) {
                const int b = wid + m * G::NWAVE;
                if (G::NYB % G::NWAVE == 0 || b < G::NYB) mfma_yblock_store<G>(Y, b, lane, ya[m], one);
            }
        }
        __syncthreads();
    });
}

}  // namespace stpi
