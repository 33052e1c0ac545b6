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
// 16 bytes of stored elements, for streaming passes.
template <class ST>
union Chunk16 {
    uint4 u;
    ST e[16 / sizeof(ST)];
};

template <class ST>
__global__ void normalize_kernel(ST *x, const ST *buf1, size_t n, const DevState *s) {
    using CT = typename Compute<ST>::type;
    constexpr int VEC = 16 / (int)sizeof(ST);
    const ST *src = s->cur ? buf1 : x;
    const CT scale = (CT)s->scale;
    const size_t stride = (size_t)gridDim.x * blockDim.x, tid = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
    size_t head = 0;
    if ((((uintptr_t)x | (uintptr_t)src) & 15) == 0) {
        // 16-byte chunks (each thread reads and writes the same chunk, so x may be src)
        const size_t nv = n / VEC;
        for (size_t i = tid; i < nv; i += stride) {
            Chunk16<ST> c;
            c.u = reinterpret_cast<const uint4 *>(src)[i];
#pragma unroll
            for (int e = 0; e < VEC; ++e) st(&c.e[e], scale * ld(&c.e[e]));
            reinterpret_cast<uint4 *>(x)[i] = c.u;
        }
        head = nv * VEC;
    }
    for (size_t i = head + tid; i < n; i += stride) st(x + i, scale * ld(src + i));
}

// Product-form chain from the caller's start x: buffer 1 <- w = f x g (as
// stored; g = 2^-2e from the bound on |f| in the state), and the state points
// at it. x itself is first overwritten by the first step.
// Also collects max |w| into the state (the first step's staging bound).
template <class ST>
__global__ void to_product_kernel(const ST *f, const ST *x, ST *w, size_t n, DevState *s) {
    using CT = typename Compute<ST>::type;
    __shared__ float red[256 / 64];
    const CT g = (CT)ldexp(1.0, -2 * bound_exponent(__uint_as_float(s->ubound), PRODUCT_ELIM));
    float m = 0.f;
    for (size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (size_t)gridDim.x * blockDim.x) {
        const CT v = (ld(f + i) * ld(x + i)) * g;
        st(w + i, v);
        m = fmaxf(m, fabsf((float)stored_value(w + i, v)));
    }
    m = block_max<256>(m, red);
    if (threadIdx.x == 0 && m > 0.f) atomicMax(&s->wmax[1], __float_as_uint(m));
    if (blockIdx.x == 0 && threadIdx.x == 0) {
        s->cur = 1;
        s->pform = 1;
    }
}

// Final pass of a product-form chain: x <- scale * (current iterate), the
// iterate being w / (f g) (0 where f = 0), computed in double as the step's
// sums are; before any step of a uniform start it is the constant 1.
template <class ST>
__global__ void from_product_kernel(ST *x, const ST *buf1, const ST *f, size_t n, const DevState *s) {
    using CT = typename Compute<ST>::type;
    constexpr int VEC = 16 / (int)sizeof(ST);
    const size_t stride = (size_t)gridDim.x * blockDim.x, tid = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (s->pform == 2) {
        const CT c = (CT)s->scale;
        for (size_t i = tid; i < n; i += stride) st(x + i, c);
        return;
    }
    const ST *src = s->cur ? buf1 : x;
    const double m = s->scale * ldexp(1.0, 2 * bound_exponent(__uint_as_float(s->ubound), PRODUCT_ELIM));
    auto one = [&](CT wv, CT fv) -> CT {
        return fv != CT(0) ? (CT)((double)wv / (double)fv * m) : CT(0);
    };
    size_t head = 0;
    if ((((uintptr_t)x | (uintptr_t)src | (uintptr_t)f) & 15) == 0) {
        // 16-byte chunks (each thread reads and writes the same chunk, so x may be src)
        const size_t nv = n / VEC;
        for (size_t i = tid; i < nv; i += stride) {
            Chunk16<ST> c, cf;
            c.u = reinterpret_cast<const uint4 *>(src)[i];
            cf.u = reinterpret_cast<const uint4 *>(f)[i];
#pragma unroll
            for (int e = 0; e < VEC; ++e) st(&c.e[e], one(ld(&c.e[e]), ld(&cf.e[e])));
            reinterpret_cast<uint4 *>(x)[i] = c.u;
        }
        head = nv * VEC;
    }
    for (size_t i = head + tid; i < n; i += stride) st(x + i, one(ld(src + i), ld(f + i)));
}

}  // namespace stpi
