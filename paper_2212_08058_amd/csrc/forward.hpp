// Forward power-iteration step and the small kernels of the iteration chain.
#pragma once

#include "stencil.hpp"

namespace stpi {

// Launch description shared by every storage type (host side).
struct FwdLaunch {
    const void *f;
    void *buf0;          // the caller's x (iterate mode: ping-pong buffer 0)
    void *buf1;          // z (iterate mode: ping-pong buffer 1)
    DevState *state;     // null: single step with x_scale, src = buf0, dst = buf1
    double x_scale;
    double *partials;    // [gridblocks][2] doubles
    int T, H, W;
    double gs[2 * 16 + 1];
    double gt[2 * 8 + 1];
};

// One variant of the step kernel: compiled radii and tile.
struct Variant {
    int RS, RT, TH, TW, NTHR, RY;
    hipError_t (*launch)(const FwdLaunch &, hipStream_t);
};

template <class ST>
struct FwdArgs {
    using CT = typename Compute<ST>::type;
    const ST *f;
    ST *buf0;
    ST *buf1;
    const DevState *state;
    double *partials;
    double x_scale;
    int T, H, W;
    Taps<CT> taps;
};

// u = f * x_stored; z = s f acc with s the scale that makes x unit;
// p1 += z * x_stored, p2 += z^2 on the values as stored. The products are
// formed in double, where they are exact for float and bfloat16 operands, so
// the residual sqrt(2 - 2 cos) keeps its accuracy near convergence.
template <class ST>
struct FwdOp {
    using CT = typename Compute<ST>::type;
    const ST *f;
    const ST *src;
    ST *dst;
    CT scale;
    __device__ __forceinline__ CT load_u(size_t i) const { return ld(f + i) * ld(src + i); }
    __device__ __forceinline__ void emit(size_t i, CT acc, double &p1, double &p2) const {
        const CT z = scale * (ld(f + i) * acc);
        st(dst + i, z);
        const double zs = (double)stored_value(dst, z);
        p2 = fma(zs, zs, p2);
        p1 = fma(zs, (double)ld(src + i), p1);
    }
};

template <class ST, int RS, int RT, int TH, int TW, int NTHR, int RY>
__global__ __launch_bounds__(NTHR) void fwd_step_kernel(FwdArgs<ST> a) {
    using CT = typename Compute<ST>::type;
    using G = Geometry<RS, RT, TH, TW, NTHR, RY>;
    __shared__ CT lds[2 * TH * G::LW];
    __shared__ double red[NTHR / 64];

    FwdOp<ST> op;
    op.f = a.f;
    if (a.state) {
        if (a.state->done) return;
        const int cur = a.state->cur;
        op.src = cur ? a.buf1 : a.buf0;
        op.dst = cur ? a.buf0 : a.buf1;
        op.scale = (CT)a.state->scale;
    } else {
        op.src = a.buf0;
        op.dst = a.buf1;
        op.scale = (CT)a.x_scale;
    }
    double d1 = 0.0, d2 = 0.0;
    const int x0 = blockIdx.x * TW, y0 = blockIdx.y * TH;
    stencil_tile<CT, RS, RT, TH, TW, NTHR, RY>(op, a.taps, a.T, a.H, a.W, x0, y0, lds, d1, d2);
    const double s1 = block_sum<NTHR>(d1, red);
    const double s2 = block_sum<NTHR>(d2, red);
    if (threadIdx.x == 0) {
        const size_t b = (size_t)blockIdx.y * gridDim.x + blockIdx.x;
        a.partials[2 * b] = s1;
        a.partials[2 * b + 1] = s2;
    }
}

template <class ST, int RS, int RT, int TH, int TW, int NTHR, int RY>
hipError_t launch_fwd(const FwdLaunch &L, hipStream_t stream) {
    using CT = typename Compute<ST>::type;
    FwdArgs<ST> a;
    a.f = (const ST *)L.f;
    a.buf0 = (ST *)L.buf0;
    a.buf1 = (ST *)L.buf1;
    a.state = L.state;
    a.partials = L.partials;
    a.x_scale = L.x_scale;
    a.T = L.T;
    a.H = L.H;
    a.W = L.W;
    // L holds taps centred at index 16 (space) and 8 (time), zero beyond the
    // problem's radii; the kernel wants them centred at its compiled RS, RT.
    for (int i = 0; i < 2 * 16 + 1; ++i) a.taps.gs[i] = CT(0);
    for (int i = 0; i < 2 * 8 + 1; ++i) a.taps.gt[i] = CT(0);
    for (int d = -RS; d <= RS; ++d) a.taps.gs[d + RS] = (CT)L.gs[d + 16];
    for (int d = -RT; d <= RT; ++d) a.taps.gt[d + RT] = (CT)L.gt[d + 8];
    dim3 grid((L.W + TW - 1) / TW, (L.H + TH - 1) / TH);
    hipLaunchKernelGGL((fwd_step_kernel<ST, RS, RT, TH, TW, NTHR, RY>), grid, dim3(NTHR), 0, stream, a);
    return hipGetLastError();
}

}  // namespace stpi
