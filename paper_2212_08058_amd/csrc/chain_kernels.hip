// Non-template kernels of the iteration chain and their host-side launchers.
#include "chain.hpp"
#include "host_internal.hpp"

namespace stpi {

__global__ void state_init_kernel(DevState *s, double scale, double tol, int max_iters) {
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
    }
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
    if (threadIdx.x == 0) {
        const double scale = s->scale;
        const double nz = sqrt(p2);
        if (!isfinite(nz) || !isfinite(p1)) {
            s->flags |= FLAG_NONFINITE;
            s->done = 1;
            return;
        }
        if (nz == 0.0) {
            s->flags |= FLAG_ZERO;
            s->done = 1;
            return;
        }
        const double c = scale * p1 / nz;
        s->rayleigh = scale * p1;
        s->lambda = nz;
        s->residual = sqrt(fmax(0.0, 2.0 - 2.0 * c));
        s->scale = 1.0 / nz;
        s->cur ^= 1;
        s->iters += 1;
        if (s->tol > 0.0 && s->residual < s->tol) {
            s->converged = 1;
            s->done = 1;
        }
        if (s->iters >= s->max_iters) s->done = 1;
    }
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

hipError_t launch_state_init(DevState *s, double scale, double tol, int max_iters, hipStream_t st) {
    hipLaunchKernelGGL(state_init_kernel, dim3(1), dim3(64), 0, st, s, scale, tol, max_iters);
    return hipGetLastError();
}

hipError_t launch_state_from_norm(const double *partials, int n, DevState *s, hipStream_t st) {
    hipLaunchKernelGGL(state_from_norm_kernel, dim3(1), dim3(CHAIN_THREADS), 0, st, partials, n, s);
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
