// Adjoint (reverse-mode) step of the normalised power iteration.
//
// Forward step k (x_k unit):  u = f x_k, v = G u, z = f v, n = ||z||,
// x_{k+1} = z / n. Given g = dL/dx_{k+1} and d = <x_{k+1}, g>:
//   g_z   = (g - x_{k+1} d) / n
//   g_u   = G (f g_z)          (G is symmetric under zero padding, so the
//                               adjoint filter is the forward stencil)
//   g_x_k = f g_u
//   g_f  += v g_z + x_k g_u
// and the epilogue accumulates <x_k, g_x_k>, the d of the next (lower) step.
// The iterates are kept unnormalised on the tape: x_k = z_k / norm_k.
#pragma once

#include "stencil.hpp"

namespace stpi {

template <class ST>
struct AdjOp {
    using CT = typename Compute<ST>::type;
    using IO = BufIO<ST>;
    static constexpr uint32_t ESZ = IO::SZ;
    const ST *f, *zk, *zk1, *vk, *g1;
    ST *gk, *gf;
    CT sk;  // 1 / norm_k
    CT c1;  // d / norm_{k+1}: x_{k+1} d = z_{k+1} c1
    CT c2;  // 1 / norm_{k+1}
    size_t plane;
    uint32_t pbytes;

    // live = false: an empty range (the loads return 0 and touch no memory)
    __device__ __forceinline__ __amdgpu_buffer_rsrc_t rs(const ST *p, int t, bool live = true) const {
        return make_rsrc(p + (size_t)(live ? t : 0) * plane, live ? pbytes : 0u);
    }

    template <int NPF>
    struct Raw {
        CT f[NPF], g[NPF], z[NPF];
    };
    template <int NPF>
    __device__ __forceinline__ void fetch(int t, const uint32_t (&off)[NPF], Raw<NPF> &raw, bool live = true) const {
        const auto rf = rs(f, t, live), rg = rs(g1, t, live), rz = rs(zk1, t, live);
#pragma unroll
        for (int k = 0; k < NPF; ++k) {
            raw.f[k] = IO::load(rf, off[k]);
            raw.g[k] = IO::load(rg, off[k]);
            raw.z[k] = IO::load(rz, off[k]);
        }
    }
    template <int NPF>
    __device__ __forceinline__ CT input(const Raw<NPF> &raw, int k) const {
        return raw.f[k] * ((raw.g[k] - raw.z[k] * c1) * c2);
    }

    template <int IPT, int QX>
    struct OutRaw {
        CT f[IPT][QX], z[IPT][QX], v[IPT][QX], g[IPT][QX], z1[IPT][QX], gf[IPT][QX];
    };
    // one element per load (a fixed count whatever the lanes)
    template <int IPT, int QX>
    __device__ __forceinline__ void fetch_out(int t, const uint32_t (&off)[IPT][QX], OutRaw<IPT, QX> &raw,
                                              bool live = true) const {
        const auto rf = rs(f, t, live), rz = rs(zk, t, live), rv = rs(vk, t, live), rg = rs(g1, t, live),
                   rz1 = rs(zk1, t, live), rgf = rs(gf, t, live);
#pragma unroll
        for (int i = 0; i < IPT; ++i)
#pragma unroll
            for (int q = 0; q < QX; ++q) {
                raw.f[i][q] = IO::load(rf, off[i][q]);
                raw.z[i][q] = IO::load(rz, off[i][q]);
                raw.v[i][q] = IO::load(rv, off[i][q]);
                raw.g[i][q] = IO::load(rg, off[i][q]);
                raw.z1[i][q] = IO::load(rz1, off[i][q]);
                raw.gf[i][q] = IO::load(rgf, off[i][q]);
            }
    }
    template <int IPT, int QX>
    __device__ __forceinline__ void emit_frame(int t, const CT (&acc)[IPT][QX], const OutRaw<IPT, QX> &raw,
                                               const uint32_t (&off)[IPT][QX], double &d1, double &d2) const {
        const auto rgk = rs(gk, t), rgf = rs(gf, t);
#pragma unroll
        for (int i = 0; i < IPT; ++i)
#pragma unroll
            for (int q = 0; q < QX; ++q) {
                const CT gu = acc[i][q];
                const CT gx = raw.f[i][q] * gu;
                const CT gz = (raw.g[i][q] - raw.z1[i][q] * c1) * c2;
                const CT xk = raw.z[i][q] * sk;
                const CT gfn = raw.gf[i][q] + raw.v[i][q] * gz + xk * gu;
                IO::store(rgk, off[i][q], gx);
                IO::store(rgf, off[i][q], gfn);
                const double gxs = (double)IO::rounded(gx);
                d1 = fma((double)xk, gxs, d1);
                d2 = fma(gxs, gxs, d2);
            }
    }
};

template <class ST>
struct AdjArgs {
    using CT = typename Compute<ST>::type;
    const ST *f, *zk, *zk1, *vk, *g1;
    ST *gk, *gf;
    const double *norm_k, *norm_k1, *d_k1;
    double *partials;
    int T, H, W, nseg;
    Taps<CT> taps;
};

template <class ST, int RS, int RT, int TH, int TW, int NTHR, int RY, int QX>
__global__ __launch_bounds__(NTHR) void adj_step_kernel(AdjArgs<ST> a) {
    using CT = typename Compute<ST>::type;
    using G = Geometry<RS, RT, TH, TW, NTHR, RY, QX>;
    __shared__ CT lds[G::LDS_ELEMS];
    __shared__ double red[NTHR / 64];
    const int nbx = (a.W + TW - 1) / TW, nby = (a.H + TH - 1) / TH;
    // work units as the forward step's: frame segments of tiles, segment-major
    const int ntiles = nbx * nby;
    const int unit = xcd_tile(blockIdx.x, ntiles * a.nseg);
    if (unit < 0) return;
    const int tile = unit % ntiles, seg = unit / ntiles;
    const int t0 = (int)((int64_t)seg * a.T / a.nseg), t1 = (int)((int64_t)(seg + 1) * a.T / a.nseg);
    AdjOp<ST> op;
    op.f = a.f;
    op.zk = a.zk;
    op.zk1 = a.zk1;
    op.vk = a.vk;
    op.g1 = a.g1;
    op.gk = a.gk;
    op.gf = a.gf;
    const double nk = *a.norm_k, nk1 = *a.norm_k1, d = *a.d_k1;
    op.sk = (CT)(1.0 / nk);
    op.c1 = (CT)(d / nk1);
    op.c2 = (CT)(1.0 / nk1);
    op.plane = (size_t)a.H * a.W;
    op.pbytes = (uint32_t)(op.plane * sizeof(ST));
    double d1 = 0.0, d2 = 0.0;
    const int x0 = (tile % nbx) * TW, y0 = (tile / nbx) * TH;
    stencil_tile<CT, RS, RT, TH, TW, NTHR, RY, QX>(op, a.taps, a.T, t0, t1, a.H, a.W, x0, y0, lds, d1, d2);
    const double s1 = block_sum<NTHR>(d1, red);
    const double s2 = block_sum<NTHR>(d2, red);
    if (threadIdx.x == 0) {
        a.partials[2 * unit] = s1;
        a.partials[2 * unit + 1] = s2;
    }
}

// Host-side description of an adjoint launch.
struct AdjLaunch {
    const void *f, *zk, *zk1, *vk, *g1;
    void *gk, *gf;
    const double *norm_k, *norm_k1, *d_k1;
    double *partials;
    int T, H, W, nseg;
    double gs[2 * 16 + 1];
    double gt[2 * 8 + 1];
};

struct AdjVariant {
    int RS, RT, TH, TW, NTHR, RY, QX;
    hipError_t (*launch)(const AdjLaunch &, hipStream_t);
};

template <class ST, int RS, int RT, int TH, int TW, int NTHR, int RY, int QX>
hipError_t launch_adj(const AdjLaunch &L, hipStream_t stream) {
    using CT = typename Compute<ST>::type;
    AdjArgs<ST> a;
    a.f = (const ST *)L.f;
    a.zk = (const ST *)L.zk;
    a.zk1 = (const ST *)L.zk1;
    a.vk = (const ST *)L.vk;
    a.g1 = (const ST *)L.g1;
    a.gk = (ST *)L.gk;
    a.gf = (ST *)L.gf;
    a.norm_k = L.norm_k;
    a.norm_k1 = L.norm_k1;
    a.d_k1 = L.d_k1;
    a.partials = L.partials;
    a.T = L.T;
    a.H = L.H;
    a.W = L.W;
    a.nseg = L.nseg > 0 ? L.nseg : 1;
    for (int i = 0; i < 2 * 16 + 1; ++i) a.taps.gs[i] = CT(0);
    for (int i = 0; i < 2 * 8 + 1; ++i) a.taps.gt[i] = CT(0);
    for (int dd = -RS; dd <= RS; ++dd) a.taps.gs[dd + RS] = (CT)L.gs[dd + 16];
    for (int dd = -RT; dd <= RT; ++dd) a.taps.gt[dd + RT] = (CT)L.gt[dd + 8];
    const int nunits = ((L.W + TW - 1) / TW) * ((L.H + TH - 1) / TH) * a.nseg;
    const int per = (nunits + NUM_XCD - 1) / NUM_XCD;
    hipLaunchKernelGGL((adj_step_kernel<ST, RS, RT, TH, TW, NTHR, RY, QX>), dim3(per * NUM_XCD), dim3(NTHR), 0,
                       stream, a);
    return hipGetLastError();
}

}  // namespace stpi
