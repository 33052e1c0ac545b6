// Non-template kernels of the iteration chain and their host-side launchers.
#include "aux.hpp"
#include "chain.hpp"
#include "host_internal.hpp"

namespace stpi {

__global__ void state_init_kernel(DevState *s, double scale, double tol, int max_iters, int check_rise, int pform) {
    if (threadIdx.x == 0 && blockIdx.x == 0) {
        s->scale = scale;
        s->residual = 0.0;
        s->lambda = 0.0;
        s->rayleigh = 0.0;
        s->tol = tol;
        s->iters = 0;
        s->done = max_iters <= 0 ? 1 : 0;
        s->cur = 0;
        s->flags = 0u;
        s->max_iters = max_iters;
        s->converged = 0;
        s->arrive = 0u;
        s->ubound = 0u;
        s->wmax[0] = s->wmax[1] = 0u;
        s->first_res[0] = s->first_res[1] = 0.0;
        s->check_rise = check_rise;
        s->pform = pform;
    }
}

// Empties the partial-sum slots of a chain whose steps finalise themselves.
__global__ void partials_empty_kernel(double *partials, int n) {
    uint64_t *w = reinterpret_cast<uint64_t *>(partials);
    for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < 2 * n; i += gridDim.x * blockDim.x)
        __hip_atomic_store(w + i, PARTIAL_EMPTY, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

__global__ void clear_word_kernel(uint32_t *w) {
    if (threadIdx.x == 0 && blockIdx.x == 0) *w = 0u;
}

// Start from the caller's vector: scale = 1 / ||x0||.
__global__ void state_from_norm_kernel(const double *partials, int n, DevState *s) {
    double ss, unused;
    sum_pairs(partials, n, ss, unused);
    if (threadIdx.x == 0) {
        const double nrm = sqrt(ss);
        if (!isfinite(nrm)) {
            s->flags |= FLAG_NONFINITE;
            s->done = 1;
        } else if (nrm == 0.0) {
            s->flags |= FLAG_ZERO;
            s->done = 1;
        } else {
            s->scale = 1.0 / nrm;
        }
    }
}

// After a step wrote z = A x_k (x_k unit) and block partials
// (sum z * x_stored, sum z^2):  n = ||z||, x_{k+1} = z / n,
// cos = <x_{k+1}, x_k> = scale * P1 / n, residual = sqrt(2 - 2 cos).
__global__ void finalize_kernel(const double *partials, int n, DevState *s) {
    if (s->done) return;
    double p1, p2;
    sum_pairs(partials, n, p1, p2);
    if (threadIdx.x == 0) step_finalize(s, p1, p2);
}

// Single-step mode: d_sums = (sum z^2, x_scale * sum z * x).
__global__ void step_sums_kernel(const double *partials, int n, double x_scale, double *d_sums) {
    double p1, p2;
    sum_pairs(partials, n, p1, p2);
    if (threadIdx.x == 0) {
        d_sums[0] = p2;
        d_sums[1] = x_scale * p1;
    }
}

// g_a_c = sum of partials; dL/dw = a (g_a - <a, g_a>)  (softmax Jacobian)
__global__ void combine_bwd_finalize(int C, int nblocks, const double *partials, const double *w, double *gw) {
    __shared__ double ga[MAX_CHANNELS];
    __shared__ double red[AUX_THREADS / 64];
    for (int c = 0; c < C; ++c) {
        double s = 0.0;
        for (int b = threadIdx.x; b < nblocks; b += AUX_THREADS) s += partials[(size_t)b * C + c];
        const double t = block_sum<AUX_THREADS>(s, red);
        if (threadIdx.x == 0) ga[c] = t;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        double a[MAX_CHANNELS];
        softmax_c(w, C, a);
        double dot = 0.0;
        for (int c = 0; c < C; ++c) dot += a[c] * ga[c];
        for (int c = 0; c < C; ++c) gw[c] = a[c] * (ga[c] - dot);
    }
}

// scalars[0] = max, scalars[1] = its first index
__global__ void max_finalize(int nblocks, const double *partials, double *scalars) {
    if (threadIdx.x != 0) return;
    double bv = -1e300, bi = 1e300;
    for (int b = 0; b < nblocks; ++b) {
        const double v = partials[2 * b], i = partials[2 * b + 1];
        if (v > bv || (v == bv && i < bi)) {
            bv = v;
            bi = i;
        }
    }
    scalars[0] = bv;
    scalars[1] = bi;
}

// out = (sum_b partials[2b]) / (a_norm ? *a_norm : 1)
__global__ void dot_finalize(const double *partials, int n, const double *a_norm, double *out) {
    double s0, s1;
    sum_pairs(partials, n, s0, s1);
    if (threadIdx.x == 0) *out = a_norm ? s0 / *a_norm : s0;
}

// out = sqrt(sum_b partials[2b + 1])  (norm of a step's output)
__global__ void norm_finalize(const double *partials, int n, double *out) {
    double s0, s1;
    sum_pairs(partials, n, s0, s1);
    if (threadIdx.x == 0) *out = sqrt(s1);
}

// out = sum_b partials[2b]  (the adjoint's <x_k, g_k>)
__global__ void sum0_finalize(const double *partials, int n, double *out) {
    double s0, s1;
    sum_pairs(partials, n, s0, s1);
    if (threadIdx.x == 0) *out = s0;
}

hipError_t launch_combine_bwd_finalize(int C, int nblocks, const double *partials, const double *w, double *gw,
                                       hipStream_t st) {
    hipLaunchKernelGGL(combine_bwd_finalize, dim3(1), dim3(AUX_THREADS), 0, st, C, nblocks, partials, w, gw);
    return hipGetLastError();
}

hipError_t launch_max_finalize(int nblocks, const double *partials, double *scalars, hipStream_t st) {
    hipLaunchKernelGGL(max_finalize, dim3(1), dim3(64), 0, st, nblocks, partials, scalars);
    return hipGetLastError();
}

hipError_t launch_dot_finalize(const double *partials, int n, const double *a_norm, double *out, hipStream_t st) {
    hipLaunchKernelGGL(dot_finalize, dim3(1), dim3(CHAIN_THREADS), 0, st, partials, n, a_norm, out);
    return hipGetLastError();
}

hipError_t launch_norm_finalize(const double *partials, int n, double *out, hipStream_t st) {
    hipLaunchKernelGGL(norm_finalize, dim3(1), dim3(CHAIN_THREADS), 0, st, partials, n, out);
    return hipGetLastError();
}

hipError_t launch_sum0_finalize(const double *partials, int n, double *out, hipStream_t st) {
    hipLaunchKernelGGL(sum0_finalize, dim3(1), dim3(CHAIN_THREADS), 0, st, partials, n, out);
    return hipGetLastError();
}

// AdamW with decoupled weight decay and optional AMSGrad on float master
// weights (Eq. 13): w <- w (1 - lr wd); m, v moment updates; vmax = max(vmax, v);
// w <- w - lr (m / bc1) / (sqrt(vmax / bc2) + eps).
template <class T>
__global__ void adamw_kernel(int64_t n, T *w, const T *g, T *m, T *v, T *vmax, T lr, T beta1, T beta2, T eps, T wd,
                             T bc1, T bc2, int amsgrad) {
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) {
        const T gi = g[i];
        T wi = w[i] * (T(1) - lr * wd);
        const T mi = beta1 * m[i] + (T(1) - beta1) * gi;
        const T vi = beta2 * v[i] + (T(1) - beta2) * gi * gi;
        T vh = vi;
        if (amsgrad) {
            vh = vmax[i] > vi ? vmax[i] : vi;
            vmax[i] = vh;
        }
        wi -= lr * (mi / bc1) / (sqrt(vh / bc2) + eps);
        m[i] = mi;
        v[i] = vi;
        w[i] = wi;
    }
}

hipError_t launch_adamw(int dtype, int64_t n, void *w, const void *g, void *m, void *v, void *vmax, double lr,
                        double beta1, double beta2, double eps, double wd, double bc1, double bc2, int amsgrad,
                        hipStream_t st) {
    const int blocks = (int)((n + 255) / 256 < 1024 ? (n + 255) / 256 : 1024);
    if (dtype == STPI_F64)
        hipLaunchKernelGGL(adamw_kernel<double>, dim3(blocks), dim3(256), 0, st, n, (double *)w, (const double *)g,
                           (double *)m, (double *)v, (double *)vmax, lr, beta1, beta2, eps, wd, bc1, bc2, amsgrad);
    else
        hipLaunchKernelGGL(adamw_kernel<float>, dim3(blocks), dim3(256), 0, st, n, (float *)w, (const float *)g,
                           (float *)m, (float *)v, (float *)vmax, (float)lr, (float)beta1, (float)beta2, (float)eps,
                           (float)wd, (float)bc1, (float)bc2, amsgrad);
    return hipGetLastError();
}

hipError_t launch_state_init(DevState *s, double scale, double tol, int max_iters, int check_rise, int pform,
                             hipStream_t st) {
    hipLaunchKernelGGL(state_init_kernel, dim3(1), dim3(64), 0, st, s, scale, tol, max_iters, check_rise, pform);
    return hipGetLastError();
}

hipError_t launch_state_from_norm(const double *partials, int n, DevState *s, hipStream_t st) {
    hipLaunchKernelGGL(state_from_norm_kernel, dim3(1), dim3(CHAIN_THREADS), 0, st, partials, n, s);
    return hipGetLastError();
}

hipError_t launch_partials_empty(double *partials, int n, hipStream_t st) {
    hipLaunchKernelGGL(partials_empty_kernel, dim3((2 * n + 255) / 256), dim3(256), 0, st, partials, n);
    return hipGetLastError();
}

hipError_t launch_clear_word(uint32_t *w, hipStream_t st) {
    hipLaunchKernelGGL(clear_word_kernel, dim3(1), dim3(64), 0, st, w);
    return hipGetLastError();
}

hipError_t launch_finalize(const double *partials, int n, DevState *s, hipStream_t st) {
    hipLaunchKernelGGL(finalize_kernel, dim3(1), dim3(CHAIN_THREADS), 0, st, partials, n, s);
    return hipGetLastError();
}

hipError_t launch_step_sums(const double *partials, int n, double x_scale, double *d_sums, hipStream_t st) {
    hipLaunchKernelGGL(step_sums_kernel, dim3(1), dim3(CHAIN_THREADS), 0, st, partials, n, x_scale, d_sums);
    return hipGetLastError();
}

}  // namespace stpi
