// Forward power-iteration step and the small kernels of the iteration chain.
#pragma once

#include <type_traits>

#include "stencil.hpp"
#include "stencil_mfma.hpp"

namespace stpi {

// Launch description shared by every storage type (host side).
struct FwdLaunch {
    const void *f;
    void *buf0;          // the caller's x (iterate mode: ping-pong buffer 0)
    void *buf1;          // z (iterate mode: ping-pong buffer 1)
    DevState *state;     // null: single step with x_scale, src = buf0, dst = buf1
    double x_scale;
    const double *norm_in;  // single step: if set, x_scale = 1 / *norm_in (read on the device)
    void *vout;             // if set, also store v = G (f x) (x unit) for the adjoint
    double *partials;    // [tiles * nseg][2] doubles
    int T, H, W;
    int nseg;            // frame segments per tile (0 is read as 1)
    int fuse;            // iterate mode: finalise the step in its last workgroup (if the variant can)
    int no_prev;         // iterate mode: the step's inner product with the previous iterate is not formed
    // matrix-core variants: float bits of a bound on |f x_stored scale| (iterate
    // mode: on |f|, the iterate being unit; single step: on |f x_stored|, scaled
    // by |x_scale| in the kernel)
    const uint32_t *ubound;
    double gs[2 * 16 + 1];
    double gt[2 * 8 + 1];
};

// One variant of the step kernel: compiled radii and tile.
using FwdLaunchFn = hipError_t (*)(const FwdLaunch &, hipStream_t);

struct Variant {
    int RS, RT, TH, TW, NTHR, RY, QX, OCC, PIPE;
    FwdLaunchFn launch;
    int (*blocks_per_cu)();  // resident workgroups per CU (occupancy query)
    FwdLaunchFn launch_p;    // product-form chain step (see FwdOpP); null where not compiled
};

template <class ST>
struct FwdArgs {
    using CT = typename Compute<ST>::type;
    const ST *f;
    ST *buf0;
    ST *buf1;
    DevState *state;
    double *partials;
    int fuse;  // 1: the last workgroup to finish reduces the partials and finalises the step
    int no_prev;  // 1: the previous iterate is not read at the outputs (p1 = 0; see FwdOp::prev)
    double x_scale;
    const double *norm_in;
    ST *vout;
    int T, H, W;
    int nseg;  // frame segments per tile: workgroup (tile, seg) owns frames [seg T / nseg, (seg + 1) T / nseg)
    const uint32_t *ubound;  // matrix-core variants (see FwdLaunch)
    int rs;                  // the problem's space radius
    Taps<CT> taps;
};

// u = f * x_stored; z = s f acc with s the scale that makes x unit;
// p1 += z * x_stored, p2 += z^2 on the values as stored. The products are
// formed in double, where they are exact for float and bfloat16 operands, so
// the residual sqrt(2 - 2 cos) keeps its accuracy near convergence.
template <class ST>
struct FwdOp {
    using CT = typename Compute<ST>::type;
    using IO = BufIO<ST>;
    static constexpr uint32_t ESZ = IO::SZ;
    const ST *f;
    const ST *src;
    ST *dst;
    ST *vout;         // optional: v = s * acc = G (f x_unit)
    CT scale;
    size_t plane;     // elements per frame
    uint32_t pbytes;  // bytes per frame
    bool cut = false;  // epilogue operands came from 4-wide loads that groups cut by the right edge extend past it
    // false: the epilogue reads the previous iterate on an empty range (as 0),
    // so p1 is 0. A chain of a fixed count of steps uses p1 (the cosine with
    // the previous iterate: the residual and the Rayleigh quotient) only on
    // its first two steps and its last; the other steps save that read.
    bool prev = true;

    template <int NPF>
    struct Raw {
        CT f[NPF], x[NPF];
    };
    // live = false issues the same loads on an empty range (they return 0 and
    // touch no memory): the matrix-core tile loop fetches every phase, so the
    // compiler's memory-counter waits count a fixed number of younger loads
    template <int NPF>
    __device__ __forceinline__ void fetch(int t, const uint32_t (&off)[NPF], Raw<NPF> &raw, bool live = true) const {
        const auto rf = make_rsrc(f + (size_t)(live ? t : 0) * plane, live ? pbytes : 0u);
        const auto rx = make_rsrc(src + (size_t)(live ? t : 0) * plane, live ? pbytes : 0u);
#pragma unroll
        for (int k = 0; k < NPF; ++k) {
            raw.f[k] = IO::load(rf, off[k]);
            raw.x[k] = IO::load(rx, off[k]);
        }
    }
    template <int NPF>
    __device__ __forceinline__ CT input(const Raw<NPF> &raw, int k) const {
        return raw.f[k] * raw.x[k];
    }
    template <int IPT, int QX>
    struct OutRaw {
        CT f[IPT][QX], x[IPT][QX];
    };
    // Epilogue operands, in a fixed count of memory instructions whatever the
    // lanes: with QX = 4 each group moves with one 4-wide access at its first
    // offset (a group cut by the right edge of the frame then reads into the
    // next row, and the epilogue, told by cut, takes f there as 0); otherwise
    // element by element. live = false issues the loads on an empty range.
    template <int IPT, int QX>
    __device__ __forceinline__ void fetch_out(int t, const uint32_t (&off)[IPT][QX], OutRaw<IPT, QX> &raw,
                                              bool live = true) const {
        const auto rf = make_rsrc(f + (size_t)(live ? t : 0) * plane, live ? pbytes : 0u);
        const auto rx = make_rsrc(src + (size_t)(live ? t : 0) * plane, live && prev ? pbytes : 0u);
#pragma unroll
        for (int i = 0; i < IPT; ++i) {
            if constexpr (QX == 4) {
                IO::load4(rf, off[i][0], raw.f[i]);
                IO::load4(rx, off[i][0], raw.x[i]);
            } else {
#pragma unroll
                for (int q = 0; q < QX; ++q) {
                    raw.f[i][q] = IO::load(rf, off[i][q]);
                    raw.x[i][q] = IO::load(rx, off[i][q]);
                }
            }
        }
    }
    // Fixed-count forms for the straight-line tile loop: every call issues the
    // same memory instructions (one per element), whatever the tile position
    // and whether the frame is emitted, so the compiler's memory-counter waits
    // never have to cover a path with fewer operations. Elements outside the
    // frame and non-emitted frames use out-of-range offsets (loads give 0,
    // stores are dropped) and add nothing to the sums.
    template <int IPT, int QX>
    __device__ __forceinline__ void fetch_out_fixed(int t, const uint32_t (&off)[IPT][QX],
                                                    OutRaw<IPT, QX> &raw) const {
        const auto rf = make_rsrc(f + (size_t)t * plane, pbytes);
        const auto rx = make_rsrc(src + (size_t)t * plane, prev ? pbytes : 0u);
#pragma unroll
        for (int i = 0; i < IPT; ++i)
#pragma unroll
            for (int q = 0; q < QX; ++q) {
                raw.f[i][q] = IO::load(rf, off[i][q]);
                raw.x[i][q] = IO::load(rx, off[i][q]);
            }
    }
    template <int IPT, int QX>
    __device__ __forceinline__ void emit_frame_fixed(int t, bool emit, const CT (&acc)[IPT][QX],
                                                     const OutRaw<IPT, QX> &raw, const uint32_t (&off)[IPT][QX],
                                                     double &d1, double &d2) const {
        const auto rz = make_rsrc(dst + (size_t)t * plane, pbytes);
        if (vout) {
            const auto rv = make_rsrc(vout + (size_t)t * plane, pbytes);
#pragma unroll
            for (int i = 0; i < IPT; ++i)
#pragma unroll
                for (int q = 0; q < QX; ++q) IO::store(rv, emit ? off[i][q] : OOB, scale * acc[i][q]);
        }
        double p1 = 0.0, p2 = 0.0;
#pragma unroll
        for (int i = 0; i < IPT; ++i)
#pragma unroll
            for (int q = 0; q < QX; ++q) {
                const CT z = scale * (raw.f[i][q] * acc[i][q]);
                const double zs = (double)IO::rounded(z);
                p2 = fma(zs, zs, p2);
                p1 = fma(zs, (double)raw.x[i][q], p1);
                IO::store(rz, emit ? off[i][q] : OOB, z);
            }
        d1 += emit ? p1 : 0.0;
        d2 += emit ? p2 : 0.0;
    }
    template <int IPT, int QX>
    __device__ __forceinline__ void emit_frame(int t, const CT (&acc)[IPT][QX], const OutRaw<IPT, QX> &raw,
                                               const uint32_t (&off)[IPT][QX], double &d1, double &d2) const {
        const auto rz = make_rsrc(dst + (size_t)t * plane, pbytes);
        if (vout) {
            const auto rv = make_rsrc(vout + (size_t)t * plane, pbytes);
#pragma unroll
            for (int i = 0; i < IPT; ++i)
#pragma unroll
                for (int q = 0; q < QX; ++q) IO::store(rv, off[i][q], scale * acc[i][q]);
        }
#pragma unroll
        for (int i = 0; i < IPT; ++i) {
            CT z[QX];
#pragma unroll
            for (int q = 0; q < QX; ++q) {
                const CT fv = cut && off[i][q] == OOB ? CT(0) : raw.f[i][q];
                z[q] = scale * (fv * acc[i][q]);
                const double zs = (double)IO::rounded(z[q]);
                d2 = fma(zs, zs, d2);
                d1 = fma(zs, (double)raw.x[i][q], d1);
            }
            if constexpr (QX == 4) {
                if (off[i][3] != OOB) {
                    IO::store4(rz, off[i][0], z);
                    continue;
                }
            }
#pragma unroll
            for (int q = 0; q < QX; ++q) IO::store(rz, off[i][q], z[q]);
        }
    }
};

// 1 / f from the hardware reciprocal (about one ulp); 0 for f = 0 and for
// subnormal f (whose outputs are negligible).
__device__ __forceinline__ float recip_or_zero(float fv) {
    return fabsf(fv) >= 1.17549435e-38f ? __builtin_amdgcn_rcpf(fv) : 0.f;
}

// Product form of a chain step (matrix-core tile loop only). The buffers hold
// w = f x g instead of the iterate x, with g = 2^-2e a power of two from the
// bound max |f| < 2^e (so w stays in range whatever the scale of f). A step
// then stages one array, w (times a power of two: w scale 2^(10 + e) =
// f x_unit 2^(10 - e)), instead of f and x, and its epilogue reads f and w at
// the outputs as the plain form reads f and x. It stores
// w_new = acc f^2 2^-S g; the iterate is w / (f g) (0 where f = 0). The
// sums are taken on its float image x~ = fl(w rcp(f)) / g: p2 = sum x~_new^2
// and p1 = sum x~_prev x~_new, products exact in double. The next step forms
// x~_prev from the same stored w and f, so it is bitwise this step's x~_new:
// the scale, the cosine and the norm all refer to one vector, which differs
// from the staged iterate by float rounding per element (the residual keeps
// float-level accuracy near convergence). The emitted sums leave out the
// powers of two 1/g: the caller multiplies d1 by ginv_in ginv_out and d2 by
// ginv_out^2. ginv_in = 1 / g of the input: 1 on the first step of a uniform
// start, whose input is f itself (w of the constant 1, up to g).
// Staging range: the staged values are w s ginv_in 2^(10 - e_in) with e_in the
// exponent of a bound on |w s ginv_in| taken from max |w| of the input buffer
// (collected by the step that wrote it; max |f| for the uniform start), so
// the largest staged value lies in [2^9, 2^10) whatever the scale of the
// iterate, and the split's half-precision parts keep their full precision
// for every value within 2^14 of it.

template <class ST>
struct FwdOpP {
    using CT = float;
    using IO = BufIO<ST>;
    static constexpr uint32_t ESZ = IO::SZ;
    const ST *f;
    const ST *src;  // w of the current iterate (or f)
    ST *dst;        // w of the next
    CT gout;        // g
    CT sg;          // 2^-S g (2^-S undoes the staging prescale): w_new = acc f^2 sg
    double ginv_in, ginv_out;
    size_t plane;
    uint32_t pbytes;
    mutable float wmax = 0.f;  // max |w_new| stored by this thread (the next step's staging bound)
    bool cut = false;          // as FwdOp::cut
    bool prev = true;          // as FwdOp::prev

    template <int NPF>
    struct Raw {
        CT u[NPF];
    };
    template <int NPF>
    __device__ __forceinline__ void fetch(int t, const uint32_t (&off)[NPF], Raw<NPF> &raw, bool live = true) const {
        const auto ru = make_rsrc(src + (size_t)(live ? t : 0) * plane, live ? pbytes : 0u);
#pragma unroll
        for (int k = 0; k < NPF; ++k) raw.u[k] = IO::load(ru, off[k]);
    }
    template <int NPF>
    __device__ __forceinline__ CT input(const Raw<NPF> &raw, int k) const {
        return raw.u[k];
    }
    template <int IPT, int QX>
    struct OutRaw {
        CT f[IPT][QX], u[IPT][QX];
    };
    template <int IPT, int QX>  // as FwdOp::fetch_out
    __device__ __forceinline__ void fetch_out(int t, const uint32_t (&off)[IPT][QX], OutRaw<IPT, QX> &raw,
                                              bool live = true) const {
        const auto rf = make_rsrc(f + (size_t)(live ? t : 0) * plane, live ? pbytes : 0u);
        const auto ru = make_rsrc(src + (size_t)(live ? t : 0) * plane, live && prev ? pbytes : 0u);
#pragma unroll
        for (int i = 0; i < IPT; ++i) {
            if constexpr (QX == 4) {
                IO::load4(rf, off[i][0], raw.f[i]);
                IO::load4(ru, off[i][0], raw.u[i]);
            } else {
#pragma unroll
                for (int q = 0; q < QX; ++q) {
                    raw.f[i][q] = IO::load(rf, off[i][q]);
                    raw.u[i][q] = IO::load(ru, off[i][q]);
                }
            }
        }
    }
    template <int IPT, int QX>
    __device__ __forceinline__ void emit_frame(int t, const CT (&acc)[IPT][QX], const OutRaw<IPT, QX> &raw,
                                               const uint32_t (&off)[IPT][QX], double &d1, double &d2) const {
        const auto rw = make_rsrc(dst + (size_t)t * plane, pbytes);
        CT wr[IPT][QX], r[IPT][QX];  // what the stores leave in memory, 1/f
#pragma unroll
        for (int i = 0; i < IPT; ++i) {
            CT w[QX];
#pragma unroll
            for (int q = 0; q < QX; ++q) {
                const CT fv = cut && off[i][q] == OOB ? CT(0) : raw.f[i][q];
                w[q] = (acc[i][q] * (fv * fv)) * sg;
                r[i][q] = recip_or_zero(fv);
            }
            bool whole = false;
            if constexpr (QX == 4) {
                if (off[i][3] != OOB) {
                    IO::store4_rounded(rw, off[i][0], w, wr[i]);
                    whole = true;
                }
            }
            if (!whole) {
#pragma unroll
                for (int q = 0; q < QX; ++q) wr[i][q] = IO::store_rounded(rw, off[i][q], w[q]);
            }
        }
        // The sums after every store of the frame: the branch on prev (uniform)
        // then holds no memory operation, so the waits that follow count the
        // same younger operations on both paths.
        if (prev) {
#pragma unroll
            for (int i = 0; i < IPT; ++i)
#pragma unroll
                for (int q = 0; q < QX; ++q) {
                    wmax = fmaxf(wmax, fabsf(wr[i][q]));
                    const double xn = (double)(wr[i][q] * r[i][q]);
                    const double xp = (double)(raw.u[i][q] * r[i][q]);
                    d2 = fma(xn, xn, d2);
                    d1 = fma(xp, xn, d1);
                }
        } else {
#pragma unroll
            for (int i = 0; i < IPT; ++i)
#pragma unroll
                for (int q = 0; q < QX; ++q) {
                    wmax = fmaxf(wmax, fabsf(wr[i][q]));
                    const double xn = (double)(wr[i][q] * r[i][q]);
                    d2 = fma(xn, xn, d2);
                }
        }
    }
};

// OCC: minimum waves per SIMD the register allocation must allow (1 = no limit;
// with NTHR = 512, OCC = 4 lets two workgroups share a CU).
// PIPE: 1 selects the software-pipelined tile loop (stencil_tile_pipe), 2 its
// straight-line form (stencil_tile_flat), 3 the matrix-core tile loop
// (stencil_tile_mfma; RS = 16, any space radius up to 16).
// PF: product-form chain step (PIPE 3, iterate mode only).
template <class ST, int RS, int RT, int TH, int TW, int NTHR, int RY, int QX, int OCC, int PIPE, bool PF>
__global__ __launch_bounds__(NTHR, OCC) void fwd_step_kernel(FwdArgs<ST> a) {
    using CT = typename Compute<ST>::type;
    using G = Geometry<RS, RT, TH, TW, NTHR, RY, QX>;
    using PG = PipeGeometry<RS, RT, TH, TW, NTHR, RY, QX>;
    static_assert(PIPE != 3 || ((RS == 16 || RS == 8) && sizeof(CT) == 4),
                  "matrix-core variants: RS 8 or 16 (the slab margin), float arithmetic");
    static_assert(!PF || PIPE == 3, "the product form runs on the matrix-core tile loop");
    constexpr int PAD = RS <= 8 ? 8 : 16;
    // bfloat16 product-form chains stage their raw bfloat16 values (one U plane)
    constexpr bool EXACT = PF && std::is_same<ST, bf16>::value;
    __shared__ CT lds[PIPE == 3 ? MfmaLds<PIPE, TH, TW, NTHR, PAD, EXACT ? 1 : 2>::value
                                : (PIPE ? PG::LDS_ELEMS : G::LDS_ELEMS)];
    __shared__ double red[NTHR / 64];

    const int nbx = (a.W + TW - 1) / TW, nby = (a.H + TH - 1) / TH;
    // consecutive units share an XCD: neighbouring tiles of one frame segment
    // (they stage overlapping slabs of the same frames at about the same time,
    // so halo lines fetched by one are L2 hits for the other)
    const int ntiles = nbx * nby;
    const int unit = xcd_tile(blockIdx.x, ntiles * a.nseg);
    if (unit < 0) return;
    const int tile = unit % ntiles, seg = unit / ntiles;
    const int t0 = (int)((int64_t)seg * a.T / a.nseg), t1 = (int)((int64_t)(seg + 1) * a.T / a.nseg);
    FwdOp<ST> op;
    op.f = a.f;
    double scale;
    if (a.state) {
        if (a.state->done) return;
        const int cur = a.state->cur;
        op.src = cur ? a.buf1 : a.buf0;
        op.dst = cur ? a.buf0 : a.buf1;
        scale = a.state->scale;
    } else {
        op.src = a.buf0;
        op.dst = a.buf1;
        scale = a.norm_in ? 1.0 / *a.norm_in : a.x_scale;
    }
    op.scale = (CT)scale;
    op.vout = a.vout;
    op.plane = (size_t)a.H * a.W;
    op.pbytes = (uint32_t)(op.plane * sizeof(ST));
    double d1 = 0.0, d2 = 0.0;
    const int x0 = (tile % nbx) * TW, y0 = (tile / nbx) * TH;
    op.cut = x0 + TW > a.W;  // 4-wide epilogue loads read past the right edge here
    op.prev = !a.no_prev;
    if constexpr (PIPE == 3) {
        // space taps centred at 16 (the kernel's are centred at RS)
        __shared__ float tapl[2 * 16 + 1];
        if (threadIdx.x < 2 * 16 + 1) {
            float g = 0.f;
#pragma unroll
            for (int i = 0; i < 2 * RS + 1; ++i) g = (int)threadIdx.x == i + 16 - RS ? (float)a.taps.gs[i] : g;
            tapl[threadIdx.x] = g;
        }
        __syncthreads();
        // staging multiplier umul = scale 2^S with |f x scale 2^S| < 2^10, output scale 2^-S
        float bound = __uint_as_float(*a.ubound);
        if constexpr (PF) {
            const int e = bound_exponent(bound, PRODUCT_ELIM);
            const bool first = a.state->pform == 2;
            const int cur = a.state->cur;
            FwdOpP<ST> pp;
            pp.f = a.f;
            pp.src = first ? a.f : op.src;
            pp.dst = op.dst;
            pp.gout = ldexpf(1.f, -2 * e);
            pp.ginv_out = ldexp(1.0, 2 * e);
            pp.ginv_in = first ? 1.0 : pp.ginv_out;
            pp.plane = op.plane;
            pp.pbytes = op.pbytes;
            pp.cut = x0 + TW > a.W;
            pp.prev = op.prev;
            // staging power of two from the input's own maximum
            const float win = first ? bound : __uint_as_float(a.state->wmax[cur]);
            float umul;
            if constexpr (EXACT) {
                // the y-pass multiplies the staged bfloat16 w by ginv_in
                // 2^(10 - ein) (a power of two, folded into its taps); the scale
                // moves to the epilogue
                const int ein = bound_exponent((float)((double)win * pp.ginv_in), 100);
                pp.sg = (float)(scale * ldexp(1.0, ein - 10 - 2 * e));
                umul = (float)ldexp(pp.ginv_in, 10 - ein);
            } else {
                const int ein = bound_exponent((float)((double)win * scale * pp.ginv_in), 100);
                pp.sg = ldexpf(1.f, ein - 10 - 2 * e);
                umul = (float)(scale * ldexp(1.0, 10 - ein) * pp.ginv_in);
            }
            stencil_tile_mfma<CT, RT, TH, TW, NTHR, PAD, EXACT>(pp, a.taps, tapl, umul, a.rs, a.T, t0, t1, a.H, a.W,
                                                          x0, y0, lds, d1, d2);
            d1 *= pp.ginv_in * pp.ginv_out;
            d2 *= pp.ginv_out * pp.ginv_out;
            const float m = block_max<NTHR>(pp.wmax, reinterpret_cast<float *>(red));
            if (threadIdx.x == 0 && m > 0.f) atomicMax(&a.state->wmax[cur ^ 1], __float_as_uint(m));
        } else {
            if (!a.state) bound *= (float)fabs(scale);
            const int e = bound_exponent(bound, 100);
            const float umul = (float)(scale * ldexp(1.0, 10 - e));
            op.scale = ldexpf(1.f, e - 10);
            stencil_tile_mfma<CT, RT, TH, TW, NTHR, PAD>(op, a.taps, tapl, umul, a.rs, a.T, t0, t1, a.H, a.W, x0, y0,
                                                   lds, d1, d2);
        }
    } else if constexpr (PIPE == 2)
        stencil_tile_flat<CT, RS, RT, TH, TW, NTHR, RY, QX>(op, a.taps, a.T, t0, t1, a.H, a.W, x0, y0, lds, d1, d2);
    else if constexpr (PIPE == 1)
        stencil_tile_pipe<CT, RS, RT, TH, TW, NTHR, RY, QX>(op, a.taps, a.T, t0, t1, a.H, a.W, x0, y0, lds, d1, d2);
    else
        stencil_tile<CT, RS, RT, TH, TW, NTHR, RY, QX>(op, a.taps, a.T, t0, t1, a.H, a.W, x0, y0, lds, d1, d2);
    const double s1 = block_sum<NTHR>(d1, red);
    const double s2 = block_sum<NTHR>(d2, red);
    __shared__ int s_last;
    if (threadIdx.x == 0) {
        if (a.fuse) {
            // Publish the two sums device-wide: agent-scope stores write through
            // the XCD's L2 into slots the last workgroup polls (PARTIAL_EMPTY);
            // the wait makes sure they are done before this workgroup is counted
            // in. Only these values cross workgroups, so no full L2 write-back is
            // needed (the kernel boundary orders the rest).
            __hip_atomic_store(&a.partials[2 * unit], s1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            __hip_atomic_store(&a.partials[2 * unit + 1], s2, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            __builtin_amdgcn_s_waitcnt(0);
            s_last = __hip_atomic_fetch_add(&a.state->arrive, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) ==
                     (unsigned)(nbx * nby * a.nseg - 1);
        } else {
            a.partials[2 * unit] = s1;
            a.partials[2 * unit + 1] = s2;
        }
    }
    if constexpr (NTHR >= FINAL_THREADS) {
        if (!a.fuse) return;
        __syncthreads();
        if (!__builtin_amdgcn_readfirstlane(s_last)) return;
        // last workgroup: the step finalisation, summed in the order of the
        // separate finalisation kernel (threads >= FINAL_THREADS add zeros);
        // agent-scope loads read the published sums past the local L2
        const int n = nbx * nby * a.nseg;
        double p1 = 0.0, p2 = 0.0;
        bool late = false;
        if (threadIdx.x < FINAL_THREADS)
            for (int i = threadIdx.x; i < n; i += FINAL_THREADS) {
                p1 += take_partial(&a.partials[2 * i], &late);
                p2 += take_partial(&a.partials[2 * i + 1], &late);
            }
        p1 = block_sum<NTHR>(p1, red);
        p2 = block_sum<NTHR>(p2, red);
        __shared__ int s_late;
        if (threadIdx.x == 0) s_late = 0;
        __syncthreads();
        if (late) s_late = 1;
        __syncthreads();
        if (threadIdx.x == 0) {
            if (s_late) a.state->flags |= FLAG_SYNC;
            step_finalize(a.state, p1, p2);
            a.state->arrive = 0u;
        }
    }
}

template <class ST, int RS, int RT, int TH, int TW, int NTHR, int RY, int QX, int OCC, int PIPE, bool PF = false>
hipError_t launch_fwd(const FwdLaunch &L, hipStream_t stream) {
    using CT = typename Compute<ST>::type;
    FwdArgs<ST> a;
    a.f = (const ST *)L.f;
    a.buf0 = (ST *)L.buf0;
    a.buf1 = (ST *)L.buf1;
    a.state = L.state;
    a.partials = L.partials;
    a.fuse = L.state && L.fuse && NTHR >= FINAL_THREADS ? 1 : 0;
    a.no_prev = L.state && L.no_prev ? 1 : 0;
    a.x_scale = L.x_scale;
    a.norm_in = L.norm_in;
    a.vout = (ST *)L.vout;
    a.T = L.T;
    a.H = L.H;
    a.W = L.W;
    a.nseg = L.nseg > 0 ? L.nseg : 1;
    a.ubound = L.ubound;
    a.rs = 0;
    for (int d = 1; d <= 16; ++d)
        if (L.gs[16 + d] != 0.0) a.rs = d;
    if (PIPE == 3 && !L.ubound) return hipErrorInvalidValue;
    if (PF && (!L.state || L.vout)) return hipErrorInvalidValue;
    // L holds taps centred at index 16 (space) and 8 (time), zero beyond the
    // problem's radii; the kernel wants them centred at its compiled RS, RT.
    for (int i = 0; i < 2 * 16 + 1; ++i) a.taps.gs[i] = CT(0);
    for (int i = 0; i < 2 * 8 + 1; ++i) a.taps.gt[i] = CT(0);
    for (int d = -RS; d <= RS; ++d) a.taps.gs[d + RS] = (CT)L.gs[d + 16];
    for (int d = -RT; d <= RT; ++d) a.taps.gt[d + RT] = (CT)L.gt[d + 8];
    const int nunits = ((L.W + TW - 1) / TW) * ((L.H + TH - 1) / TH) * a.nseg;
    const int per = (nunits + NUM_XCD - 1) / NUM_XCD;
    hipLaunchKernelGGL((fwd_step_kernel<ST, RS, RT, TH, TW, NTHR, RY, QX, OCC, PIPE, PF>), dim3(per * NUM_XCD),
                       dim3(NTHR), 0, stream, a);
    return hipGetLastError();
}

template <int NTHR>
constexpr bool fwd_can_fuse() {
    return NTHR >= FINAL_THREADS;
}

// Matrix-core variants report the occupancy of their product-form kernel,
// the one an iteration chain runs (with bfloat16 storage it stages a single
// half plane and may fit more workgroups per CU than the plain step).
template <class ST, int RS, int RT, int TH, int TW, int NTHR, int RY, int QX, int OCC, int PIPE>
int fwd_blocks_per_cu() {
    int n = 0;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(
            &n, fwd_step_kernel<ST, RS, RT, TH, TW, NTHR, RY, QX, OCC, PIPE, PIPE == 3>, NTHR, 0) != hipSuccess)
        n = 1;
    return n > 0 ? n : 1;
}

// The product-form launcher of a variant (matrix-core variants only).
template <class ST, int RS, int RT, int TH, int TW, int NTHR, int RY, int QX, int OCC, int PIPE>
constexpr FwdLaunchFn product_launcher() {
    if constexpr (PIPE == 3)
        return &launch_fwd<ST, RS, RT, TH, TW, NTHR, RY, QX, OCC, PIPE, true>;
    else
        return nullptr;
}

}  // namespace stpi
