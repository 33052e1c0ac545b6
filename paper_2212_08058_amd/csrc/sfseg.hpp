// Full SFSeg step (Sec. 3, Eq. 7 / Eq. 10): the update with the first-order
// Taylor affinity of Eq. 2,
//
//   z = s (1/alpha - f^2) G*(s x) - s G*(f^2 s x) + 2 s f G*(f s x),
//
// i.e. z_i = s_i sum_j s_j [1/alpha - (f_i - f_j)^2] G_ij x_j, with s the unary
// map raised to p and f the pairwise feature. The three filtered fields go
// through one separable stencil pass: a workgroup owns a TH x TW output tile
// and streams its frames; per frame it stages u1 = s x, u2 = f^2 s x and
// u3 = f s x on the halo-extended tile into three LDS planes (one load of s,
// f and x per element, issued a frame ahead), runs the y-pass and the x-pass
// on each plane, scatters the three results into three register rings of
// 2 RT + 1 output frames (the t-pass), and recombines them per output voxel
// with that voxel's own s and f. Zero padding comes from out-of-range buffer
// loads, as in the single-field step. The reduction partials (sum z^2 and
// sum z x_stored) and the last-workgroup finalisation are those of the
// single-field step kernel.
#pragma once

#include "stencil.hpp"

namespace stpi {

template <class ST>
struct SfsegArgs {
    using CT = typename Compute<ST>::type;
    const ST *s;  // unary map to the power p
    const ST *f;  // pairwise feature
    ST *buf0;
    ST *buf1;
    DevState *state;  // null: single step (src = buf0, dst = buf1, scale x_scale)
    double *partials;
    int fuse;
    double x_scale;
    CT ainv;  // 1 / alpha
    int T, H, W;
    int nseg;
    Taps<CT> taps;
};

template <int RS, int RT, int TH, int TW, int NTHR, int RY, int QX>
struct SfsegGeometry {
    using G = Geometry<RS, RT, TH, TW, NTHR, RY, QX>;
    static constexpr int PLANE = G::LDS_ELEMS;  // one field: staged tile, then the y-pass output
    static constexpr int LDS_ELEMS = 3 * PLANE;
};

template <class ST, int RS, int RT, int TH, int TW, int NTHR, int RY, int QX>
__global__ __launch_bounds__(NTHR) void sfseg_step_kernel(SfsegArgs<ST> a) {
    using CT = typename Compute<ST>::type;
    using IO = BufIO<ST>;
    using G = Geometry<RS, RT, TH, TW, NTHR, RY, QX>;
    using SG = SfsegGeometry<RS, RT, TH, TW, NTHR, RY, QX>;
    constexpr int NC = G::NC, NU = G::NU, NPF = G::NPF, LW = G::LW, RSA = G::RSA;
    constexpr int NYI = G::NYI, NQ = G::NQ, NXI = G::NXI, IPT = G::IPT, NTS = G::NTS;
    constexpr uint32_t ESZ = IO::SZ;
    __shared__ CT lds[SG::LDS_ELEMS];
    __shared__ double red[NTHR / 64];

    const int nbx = (a.W + TW - 1) / TW, nby = (a.H + TH - 1) / TH;
    const int unit = xcd_tile(blockIdx.x, nbx * nby * a.nseg);
    if (unit < 0) return;
    const int tile = unit / a.nseg, seg = unit % a.nseg;
    const int t0 = (int)((int64_t)seg * a.T / a.nseg), t1 = (int)((int64_t)(seg + 1) * a.T / a.nseg);
    const ST *src;
    ST *dst;
    double scale;
    if (a.state) {
        if (a.state->done) return;
        const int cur = a.state->cur;
        src = cur ? a.buf1 : a.buf0;
        dst = cur ? a.buf0 : a.buf1;
        scale = a.state->scale;
    } else {
        src = a.buf0;
        dst = a.buf1;
        scale = a.x_scale;
    }
    const CT sc = (CT)scale;
    const size_t plane = (size_t)a.H * a.W;
    const uint32_t pbytes = (uint32_t)(plane * ESZ);
    const int x0 = (tile % nbx) * TW, y0 = (tile / nbx) * TH;
    const int tid = threadIdx.x;
    const Taps<CT> &tp = a.taps;

    // staged-element offsets, as in the single-field plain tile loop
    uint32_t poff[NPF];
#pragma unroll
    for (int k = 0; k < NPF; ++k) {
        const int e = tid + k * NTHR;
        const int r = e / NC, c = e % NC;
        const int gy = y0 - RS + r, gx = x0 - RS + c;
        const bool ok = e < NU && (unsigned)gy < (unsigned)a.H && (unsigned)gx < (unsigned)a.W;
        poff[k] = ok ? (uint32_t)(gy * a.W + gx) * ESZ : OOB;
    }
    uint32_t ooff[IPT][QX];
    int orow[IPT], ocol[IPT];
#pragma unroll
    for (int i = 0; i < IPT; ++i) {
        const int item = tid + i * NTHR;
        const bool live = item < NXI;
        orow[i] = live ? item / NQ : 0;
        ocol[i] = live ? (item % NQ) * QX : 0;
#pragma unroll
        for (int q = 0; q < QX; ++q) {
            const int gy = y0 + orow[i], gx = x0 + ocol[i] + q;
            ooff[i][q] = (live && gy < a.H && gx < a.W) ? (uint32_t)(gy * a.W + gx) * ESZ : OOB;
        }
    }

    CT acc[3][NTS][IPT][QX];
#pragma unroll
    for (int m = 0; m < 3; ++m)
#pragma unroll
        for (int s = 0; s < NTS; ++s)
#pragma unroll
            for (int i = 0; i < IPT; ++i)
#pragma unroll
                for (int q = 0; q < QX; ++q) acc[m][s][i][q] = CT(0);

    const FrameWalk<RT> fw(a.T, t0, t1);  // frame order (the last segment walks backward)
    CT ps[NPF], pfv[NPF], px[NPF];
    // ok = false issues the same loads on an empty range (they return 0 and
    // touch no memory): both load groups below are issued in every frame, so
    // the compiler's memory-counter waits before each use allow for the
    // younger group instead of draining it
    auto fetch = [&](int t, bool ok) __attribute__((always_inline)) {
        const size_t tt = ok ? (size_t)t : 0;
        const uint32_t pb = ok ? pbytes : 0u;
        const auto rs = make_rsrc(a.s + tt * plane, pb);
        const auto rf = make_rsrc(a.f + tt * plane, pb);
        const auto rx = make_rsrc(src + tt * plane, pb);
#pragma unroll
        for (int k = 0; k < NPF; ++k) {
            ps[k] = IO::load(rs, poff[k]);
            pfv[k] = IO::load(rf, poff[k]);
            px[k] = IO::load(rx, poff[k]);
        }
    };
    fetch(fw.in(0), true);
    CT os[IPT][QX], of[IPT][QX], ox[IPT][QX];
    double d1 = 0.0, d2 = 0.0;

    ring_loop<NTS, 0>(fw.nstep, [&](auto ring_pos, int i) __attribute__((always_inline)) {
        constexpr int J = decltype(ring_pos)::value;
        CT v[3][IPT][QX];
        const bool live = i < fw.nin;
        const int tout = fw.out(i);
        const bool emit = tout >= t0 && tout < t1;
        {
            // the epilogue's operands (empty range when the frame is not emitted)
            const size_t to = emit ? (size_t)tout : 0;
            const uint32_t pb = emit ? pbytes : 0u;
            const auto rs = make_rsrc(a.s + to * plane, pb);
            const auto rf = make_rsrc(a.f + to * plane, pb);
            const auto rx = make_rsrc(src + to * plane, pb);
#pragma unroll
            for (int ii = 0; ii < IPT; ++ii)
#pragma unroll
                for (int q = 0; q < QX; ++q) {
                    os[ii][q] = IO::load(rs, ooff[ii][q]);
                    of[ii][q] = IO::load(rf, ooff[ii][q]);
                    ox[ii][q] = IO::load(rx, ooff[ii][q]);
                }
        }
        if (live) {
            // stage the three fields of this frame
#pragma unroll
            for (int k = 0; k < NPF; ++k) {
                const int e = tid + k * NTHR;
                if (NU % NTHR == 0 || k < NPF - 1 || e < NU) {
                    const CT u1 = (ps[k] * px[k]) * sc;
                    const CT u3 = pfv[k] * u1;
                    lds[e] = u1;
                    lds[SG::PLANE + e] = pfv[k] * u3;
                    lds[2 * SG::PLANE + e] = u3;
                }
            }
        }
        fetch(fw.in(i + 1), i + 1 < fw.nin);
        if (live) {
            __syncthreads();
            // y-pass of each field: RY rows of one halo column per item
            for (int it = tid; it < NYI; it += NTHR) {
                const int c = it % NC;
                const int g = it / NC;
#pragma unroll
                for (int m = 0; m < 3; ++m) {
                    const CT *col = lds + m * SG::PLANE + (g * RY) * NC + c;
                    CT u[RY + 2 * RS];
#pragma unroll
                    for (int k = 0; k < RY + 2 * RS; ++k) u[k] = col[k * NC];
                    CT *dstp = lds + m * SG::PLANE + G::NUP + (g * RY) * LW + c + (RSA - RS);
#pragma unroll
                    for (int r = 0; r < RY; ++r) {
                        CT sum = CT(0);
#pragma unroll
                        for (int d = 0; d <= 2 * RS; ++d) sum = fma(tp.gs[d], u[r + d], sum);
                        dstp[r * LW] = sum;
                    }
                }
            }
            __syncthreads();
            // x-pass of each field: QX outputs of a row per item, 16-byte LDS reads
#pragma unroll
            for (int ii = 0; ii < IPT; ++ii) {
                using V4 = LdsVec<CT>;
                constexpr int NV = (QX + 2 * RSA) / V4::N;
#pragma unroll
                for (int m = 0; m < 3; ++m) {
                    const typename V4::type *rowp = reinterpret_cast<const typename V4::type *>(
                        __builtin_assume_aligned(lds + m * SG::PLANE + G::NUP + orow[ii] * LW + ocol[ii], 16));
                    CT w[QX + 2 * RSA];
#pragma unroll
                    for (int k = 0; k < NV; ++k) {
                        const typename V4::type t = rowp[k];
#pragma unroll
                        for (int e = 0; e < V4::N; ++e) w[k * V4::N + e] = t[e];
                    }
#pragma unroll
                    for (int q = 0; q < QX; ++q) {
                        CT sum = CT(0);
#pragma unroll
                        for (int d = 0; d <= 2 * RS; ++d) sum = fma(tp.gs[d], w[q + d + RSA - RS], sum);
                        v[m][ii][q] = sum;
                    }
                }
            }
            // t-pass: each field's ring
#pragma unroll
            for (int m = 0; m < 3; ++m) ring_scatter<J, -RT, RT>(acc[m], v[m], tp);
        }
        constexpr int es = ((J - RT) % NTS + NTS) % NTS;
        if (emit) {
            const auto rz = make_rsrc(dst + (size_t)tout * plane, pbytes);
#pragma unroll
            for (int ii = 0; ii < IPT; ++ii)
#pragma unroll
                for (int q = 0; q < QX; ++q) {
                    const CT fo = of[ii][q];
                    const CT A = acc[0][es][ii][q], B = acc[1][es][ii][q], C = acc[2][es][ii][q];
                    const CT z = os[ii][q] * (fma(a.ainv - fo * fo, A, -B) + CT(2) * fo * C);
                    const double zs = (double)IO::rounded(z);
                    d2 = fma(zs, zs, d2);
                    d1 = fma(zs, (double)ox[ii][q], d1);
                    IO::store(rz, ooff[ii][q], z);
                }
        }
#pragma unroll
        for (int m = 0; m < 3; ++m)
#pragma unroll
            for (int ii = 0; ii < IPT; ++ii)
#pragma unroll
                for (int q = 0; q < QX; ++q) acc[m][es][ii][q] = CT(0);
    });

    const double s1 = block_sum<NTHR>(d1, red);
    const double s2 = block_sum<NTHR>(d2, red);
    __shared__ int s_last;
    if (threadIdx.x == 0) {
        if (a.fuse) {
            // as the single-field step: write-through publication, polled slots
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

// The range check of the affinity (Eq. 2's Taylor term): every entry of M is
// >= 0 when s >= 0 and alpha (max f - min f)^2 <= 1. Per-block min f, max f,
// min s into partials[3 b .. 3 b + 2].
constexpr int SFSEG_RANGE_BLOCKS = 256;
template <class ST>
__global__ void sfseg_range_kernel(size_t n, const ST *s, const ST *f, double *partials) {
    using CT = typename Compute<ST>::type;
    __shared__ double r0[256 / 64], r1[256 / 64], r2[256 / 64];
    double fmn = INFINITY, fmx = -INFINITY, smn = INFINITY;
    for (size_t i = (size_t)blockIdx.x * 256 + threadIdx.x; i < n; i += (size_t)gridDim.x * 256) {
        const double fv = (double)ld(f + i), sv = (double)ld(s + i);
        // a NaN makes the check fail
        fmn = (fv < fmn || fv != fv) ? fv : fmn;
        fmx = (fv > fmx || fv != fv) ? fv : fmx;
        smn = (sv < smn || sv != sv) ? sv : smn;
    }
#pragma unroll
    for (int off = 32; off >= 1; off >>= 1) {
        const double a = __shfl_xor(fmn, off, 64), b = __shfl_xor(fmx, off, 64), c = __shfl_xor(smn, off, 64);
        fmn = (a < fmn || a != a) ? a : fmn;
        fmx = (b > fmx || b != b) ? b : fmx;
        smn = (c < smn || c != c) ? c : smn;
    }
    const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
    if (lane == 0) {
        r0[wid] = fmn;
        r1[wid] = fmx;
        r2[wid] = smn;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        for (int w = 1; w < 256 / 64; ++w) {
            fmn = (r0[w] < fmn || r0[w] != r0[w]) ? r0[w] : fmn;
            fmx = (r1[w] > fmx || r1[w] != r1[w]) ? r1[w] : fmx;
            smn = (r2[w] < smn || r2[w] != r2[w]) ? r2[w] : smn;
        }
        partials[3 * blockIdx.x] = fmn;
        partials[3 * blockIdx.x + 1] = fmx;
        partials[3 * blockIdx.x + 2] = smn;
    }
}

template <class ST>
__global__ void sfseg_unary_kernel(size_t n, const ST *S, double p, ST *s) {
    using CT = typename Compute<ST>::type;
    for (size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (size_t)gridDim.x * blockDim.x) {
        const CT v = ld(S + i);
        // S^p for S >= 0 (0^p = 0 for p > 0, 1 for p = 0); NaN for negative S
        st(s + i, (CT)pow((double)v, p));
    }
}

struct SfsegLaunch {
    const void *s, *f;
    void *buf0, *buf1;
    DevState *state;
    double *partials;
    int fuse;
    double x_scale;
    double ainv;
    int T, H, W, nseg;
    double gs[2 * 16 + 1];
    double gt[2 * 8 + 1];
};

using SfsegLaunchFn = hipError_t (*)(const SfsegLaunch &, hipStream_t);

struct SfsegVariant {
    int RS, RT, TH, TW, NTHR;
    SfsegLaunchFn launch;
    int (*blocks_per_cu)();
};

template <class ST, int RS, int RT, int TH, int TW, int NTHR, int RY, int QX>
hipError_t launch_sfseg(const SfsegLaunch &L, hipStream_t stream) {
    using CT = typename Compute<ST>::type;
    SfsegArgs<ST> a;
    a.s = (const ST *)L.s;
    a.f = (const ST *)L.f;
    a.buf0 = (ST *)L.buf0;
    a.buf1 = (ST *)L.buf1;
    a.state = L.state;
    a.partials = L.partials;
    a.fuse = L.state && L.fuse && NTHR >= FINAL_THREADS ? 1 : 0;
    a.x_scale = L.x_scale;
    a.ainv = (CT)L.ainv;
    a.T = L.T;
    a.H = L.H;
    a.W = L.W;
    a.nseg = L.nseg > 0 ? L.nseg : 1;
    for (int i = 0; i < 2 * 16 + 1; ++i) a.taps.gs[i] = CT(0);
    for (int i = 0; i < 2 * 8 + 1; ++i) a.taps.gt[i] = CT(0);
    for (int d = -RS; d <= RS; ++d) a.taps.gs[d + RS] = (CT)L.gs[d + 16];
    for (int d = -RT; d <= RT; ++d) a.taps.gt[d + RT] = (CT)L.gt[d + 8];
    const int nunits = ((L.W + TW - 1) / TW) * ((L.H + TH - 1) / TH) * a.nseg;
    const int per = (nunits + NUM_XCD - 1) / NUM_XCD;
    hipLaunchKernelGGL((sfseg_step_kernel<ST, RS, RT, TH, TW, NTHR, RY, QX>), dim3(per * NUM_XCD), dim3(NTHR), 0,
                       stream, a);
    return hipGetLastError();
}

template <class ST, int RS, int RT, int TH, int TW, int NTHR, int RY, int QX>
int sfseg_blocks_per_cu() {
    int n = 0;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&n, sfseg_step_kernel<ST, RS, RT, TH, TW, NTHR, RY, QX>, NTHR,
                                                     0) != hipSuccess)
        n = 1;
    return n > 0 ? n : 1;
}

}  // namespace stpi
