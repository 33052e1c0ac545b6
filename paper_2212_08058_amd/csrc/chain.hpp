// Small kernels around the step: start vector, norm reduction, per-step
// finalisation (Eq. 8 normalisation factor, residual, stopping) and the final
// normalisation pass. All reductions run in double, in a fixed order.
#pragma once

#include "common.hpp"

namespace stpi {

constexpr int CHAIN_THREADS = FINAL_THREADS;
constexpr int NORM_BLOCKS = 512;  // fixed grid for the sum-of-squares pass

// Sums partials[2*i + k] over i in [0, n) for k = 0, 1 (one workgroup).
__device__ __forceinline__ void sum_pairs(const double *partials, int n, double &s0, double &s1) {
    __shared__ double red[CHAIN_THREADS / 64];
    double a = 0.0, b = 0.0;
    for (int i = threadIdx.x; i < n; i += CHAIN_THREADS) {
        a += partials[2 * i];
        b += partials[2 * i + 1];
    }
    s0 = block_sum<CHAIN_THREADS>(a, red);
    s1 = block_sum<CHAIN_THREADS>(b, red);
}

template <class ST>
__global__ void fill_ones_kernel(ST *x, size_t n) {
    using CT = typename Compute<ST>::type;
    for (size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (size_t)gridDim.x * blockDim.x)
        st(x + i, CT(1));
}

template <class ST>
__global__ void sumsq_kernel(const ST *x, size_t n, double *partials) {
    __shared__ double red[CHAIN_THREADS / 64];
    double a = 0.0;
    for (size_t i = (size_t)blockIdx.x * CHAIN_THREADS + threadIdx.x; i < n; i += (size_t)gridDim.x * CHAIN_THREADS) {
        const double v = (double)ld(x + i);
        a += v * v;
    }
    const double s = block_sum<CHAIN_THREADS>(a, red);
    if (threadIdx.x == 0) {
        partials[2 * blockIdx.x] = s;
        partials[2 * blockIdx.x + 1] = 0.0;
    }
}

// x <- scale * (current iterate), written into the caller's buffer.
template <class ST>
__global__ void normalize_kernel(ST *x, const ST *buf1, size_t n, const DevState *s) {
    using CT = typename Compute<ST>::type;
    const ST *src = s->cur ? buf1 : x;
    const CT scale = (CT)s->scale;
    for (size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (size_t)gridDim.x * blockDim.x)
        st(x + i, scale * ld(src + i));
}

}  // namespace stpi
