// Element-wise and reduction kernels around the iteration: channel
// combination (forward/backward), normalisation by a device norm, inner
// products, and the BCE loss with its gradient. All reductions use fixed-order
// double sums (per-thread, wavefront shuffle, workgroup, then one finalising
// workgroup), so results are bitwise reproducible.
#pragma once

#include "chain.hpp"
#include "stencil.hpp"

namespace stpi {

constexpr int AUX_THREADS = 256;
constexpr int AUX_BLOCKS = 512;
constexpr int MAX_CHANNELS = 64;
constexpr double BCE_EPS = 1e-7;

// softmax(w) over C <= MAX_CHANNELS logits, in double (each workgroup
// recomputes it; C is tiny).
__device__ __forceinline__ void softmax_c(const double *w, int C, double *a) {
    double m = -1e300;
    for (int c = 0; c < C; ++c) m = fmax(m, (double)w[c]);
    double s = 0.0;
    for (int c = 0; c < C; ++c) {
        a[c] = exp((double)w[c] - m);
        s += a[c];
    }
    for (int c = 0; c < C; ++c) a[c] /= s;
}

// f = sum_c softmax(w)_c fc[c]   (fc is [C][n])
template <class ST>
__global__ void combine_fwd_kernel(int C, size_t n, const ST *fc, const double *w, ST *f) {
    using CT = typename Compute<ST>::type;
    __shared__ double a_s[MAX_CHANNELS];
    if (threadIdx.x == 0) softmax_c(w, C, a_s);
    __syncthreads();
    for (size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (size_t)gridDim.x * blockDim.x) {
        CT s = CT(0);
        for (int c = 0; c < C; ++c) s = fma((CT)a_s[c], ld(fc + (size_t)c * n + i), s);
        st(f + i, s);
    }
}

// partials[b*C + c] = sum over this workgroup's elements of g_f * fc[c]
template <class ST>
__global__ void combine_bwd_kernel(int C, size_t n, const ST *fc, const ST *gf, double *partials) {
    __shared__ double red[AUX_THREADS / 64];
    for (int c = 0; c < C; ++c) {
        double s = 0.0;
        for (size_t i = (size_t)blockIdx.x * AUX_THREADS + threadIdx.x; i < n; i += (size_t)gridDim.x * AUX_THREADS)
            s = fma((double)ld(gf + i), (double)ld(fc + (size_t)c * n + i), s);
        const double t = block_sum<AUX_THREADS>(s, red);
        if (threadIdx.x == 0) partials[(size_t)blockIdx.x * C + c] = t;
    }
}

// x = z / norm
template <class ST>
__global__ void scale_by_norm_kernel(size_t n, const ST *z, const double *norm, ST *x) {
    using CT = typename Compute<ST>::type;
    const CT s = (CT)(1.0 / *norm);
    for (size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (size_t)gridDim.x * blockDim.x)
        st(x + i, ld(z + i) * s);
}

// partials[2b] = sum a * b over the workgroup's elements (exact double products)
template <class ST>
__global__ void dot_kernel(size_t n, const ST *a, const ST *b, double *partials) {
    __shared__ double red[AUX_THREADS / 64];
    double s = 0.0;
    for (size_t i = (size_t)blockIdx.x * AUX_THREADS + threadIdx.x; i < n; i += (size_t)gridDim.x * AUX_THREADS)
        s = fma((double)ld(a + i), (double)ld(b + i), s);
    const double t = block_sum<AUX_THREADS>(s, red);
    if (threadIdx.x == 0) {
        partials[2 * blockIdx.x] = t;
        partials[2 * blockIdx.x + 1] = 0.0;
    }
}

// Fills x with 1 and sets norm = sqrt(n) (the uniform start x0 = 1 / sqrt(N)).
template <class ST>
__global__ void train_init_kernel(size_t n, ST *x, double *norm) {
    using CT = typename Compute<ST>::type;
    if (blockIdx.x == 0 && threadIdx.x == 0) *norm = sqrt((double)n);
    for (size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (size_t)gridDim.x * blockDim.x)
        st(x + i, CT(1));
}

// Per-workgroup maximum and its first index: partials[2b] = max, [2b+1] = index.
// *out = max(*out, max_i |f_i| (x null) or |f_i x_i|) as float bits (the
// values are >= 0, so their bit patterns order as the floats do; NaNs are
// skipped). The bound that scales the matrix-core step's half-precision
// operands.
template <class ST>
__global__ void bound_kernel(size_t n, const ST *f, const ST *x, uint32_t *out) {
    __shared__ float red[AUX_THREADS / 64];
    constexpr int VEC = 16 / (int)sizeof(ST);
    float r = 0.f;
    const size_t stride = (size_t)gridDim.x * AUX_THREADS, tid = (size_t)blockIdx.x * AUX_THREADS + threadIdx.x;
    size_t head = 0;
    if ((((uintptr_t)f | (uintptr_t)x) & 15) == 0) {
        // 16-byte chunks, four independent loads in flight per thread
        const size_t nv = n / VEC;
        const uint4 *f4 = reinterpret_cast<const uint4 *>(f), *x4 = reinterpret_cast<const uint4 *>(x);
        auto take = [&](const Chunk16<ST> &cf, const Chunk16<ST> &cx) __attribute__((always_inline)) {
#pragma unroll
            for (int e = 0; e < VEC; ++e) {
                float v = fabsf((float)ld(&cf.e[e]));
                if (x) v *= fabsf((float)ld(&cx.e[e]));
                r = v > r ? v : r;
            }
        };
        constexpr int U = 4;
        size_t i = tid;
        for (; i + (U - 1) * stride < nv; i += U * stride) {
            Chunk16<ST> cf[U], cx[U];
#pragma unroll
            for (int k = 0; k < U; ++k) {
                cf[k].u = f4[i + k * stride];
                if (x) cx[k].u = x4[i + k * stride];
            }
#pragma unroll
            for (int k = 0; k < U; ++k) take(cf[k], cx[k]);
        }
        for (; i < nv; i += stride) {
            Chunk16<ST> cf, cx;
            cf.u = f4[i];
            if (x) cx.u = x4[i];
            take(cf, cx);
        }
        head = nv * VEC;
    }
    for (size_t i = head + tid; i < n; i += stride) {
        float v = fabsf((float)ld(f + i));
        if (x) v *= fabsf((float)ld(x + i));
        r = v > r ? v : r;
    }
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) {
        const float w = __shfl_xor(r, o, 64);
        r = w > r ? w : r;
    }
    if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = r;
    __syncthreads();
    if (threadIdx.x == 0) {
        for (int w = 1; w < AUX_THREADS / 64; ++w) r = red[w] > r ? red[w] : r;
        // only workgroups that raise the maximum touch it: thousands of
        // atomics on one word would serialise
        const uint32_t cur = __hip_atomic_load(out, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        if (__float_as_uint(r) > cur) atomicMax(out, __float_as_uint(r));
    }
}

template <class ST>
__global__ void max_kernel(size_t n, const ST *x, double *partials) {
    __shared__ double sv[AUX_THREADS];
    __shared__ double si[AUX_THREADS];
    double bv = -1e300, bi = 1e300;
    for (size_t i = (size_t)blockIdx.x * AUX_THREADS + threadIdx.x; i < n; i += (size_t)gridDim.x * AUX_THREADS) {
        const double v = (double)ld(x + i);
        if (v > bv) {
            bv = v;
            bi = (double)i;
        }
    }
    sv[threadIdx.x] = bv;
    si[threadIdx.x] = bi;
    __syncthreads();
    for (int s = AUX_THREADS / 2; s > 0; s >>= 1) {
        if ((int)threadIdx.x < s) {
            const double ov = sv[threadIdx.x + s], oi = si[threadIdx.x + s];
            if (ov > sv[threadIdx.x] || (ov == sv[threadIdx.x] && oi < si[threadIdx.x])) {
                sv[threadIdx.x] = ov;
                si[threadIdx.x] = oi;
            }
        }
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        partials[2 * blockIdx.x] = sv[0];
        partials[2 * blockIdx.x + 1] = si[0];
    }
}

// y = clip(x / m, eps, 1 - eps); loss_i = -(g log y + (1-g) log(1-y));
// g_y = (y - g) / (y (1 - y)) / n where not clipped, else 0; g_x = g_y / m.
// partials[2b] = sum loss_i, [2b+1] = sum g_y x.
template <class ST>
__global__ void bce_kernel(size_t n, const ST *x, const uint8_t *gt, const double *scalars, ST *gx,
                           double *partials) {
    __shared__ double red[AUX_THREADS / 64];
    const double m = scalars[0];
    const double inv_n = 1.0 / (double)n;
    double sl = 0.0, sg = 0.0;
    for (size_t i = (size_t)blockIdx.x * AUX_THREADS + threadIdx.x; i < n; i += (size_t)gridDim.x * AUX_THREADS) {
        const double xv = (double)ld(x + i);
        const double g = gt[i] ? 1.0 : 0.0;
        const double yr = xv / m;
        const double y = fmin(fmax(yr, BCE_EPS), 1.0 - BCE_EPS);
        sl -= g * log(y) + (1.0 - g) * log(1.0 - y);
        const double gy = (yr > BCE_EPS && yr < 1.0 - BCE_EPS) ? (y - g) / (y * (1.0 - y)) * inv_n : 0.0;
        sg = fma(gy, xv, sg);
        st(gx + i, (typename Compute<ST>::type)(gy / m));
    }
    const double a = block_sum<AUX_THREADS>(sl, red);
    const double b = block_sum<AUX_THREADS>(sg, red);
    if (threadIdx.x == 0) {
        partials[2 * blockIdx.x] = a;
        partials[2 * blockIdx.x + 1] = b;
    }
}

// loss = sum loss_i / n; the max-normalisation term of the derivative goes to
// the first argmax: g_x[a] -= sum(g_y x) / m^2.
template <class ST>
__global__ void bce_finalize(size_t n, int nblocks, const double *partials, const double *scalars, ST *gx,
                             double *loss) {
    double a, b;
    sum_pairs(partials, nblocks, a, b);
    if (threadIdx.x == 0) {
        const double m = scalars[0];
        const size_t am = (size_t)scalars[1];
        *loss = a / (double)n;
        st(gx + am, (typename Compute<ST>::type)((double)ld(gx + am) - b / (m * m)));
    }
}

}  // namespace stpi
