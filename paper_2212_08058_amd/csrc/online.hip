// Online / partial iteration over video sub-windows (Sec. 4, "Online vs
// Offline processing"): the start vector of a q-frame window from the final
// solution of the previous window, which lies `shift` frames earlier.
#include <hip/hip_runtime.h>

#include <cmath>

#include "../../include/stpi.h"
#include "common.hpp"
#include "host_internal.hpp"

namespace stpi {
namespace {

// x0[t] = x_prev[t + shift] for t < q - shift (the overlapping frames), and
// the uniform start value c for the `shift` new frames.
template <class ST>
__global__ void window_start_kernel(const ST *x_prev, ST *x0, size_t plane, int q, int shift, double c) {
    using CT = typename Compute<ST>::type;
    const size_t n = plane * (size_t)q, keep = plane * (size_t)(q - shift), off = plane * (size_t)shift;
    for (size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (size_t)gridDim.x * blockDim.x)
        st(x0 + i, i < keep ? (CT)ld(x_prev + i + off) : (CT)c);
}

}  // namespace
}  // namespace stpi

using namespace stpi;

extern "C" {

int stpi_window_start(const stpi_problem *pw, const void *x_prev, int shift, void *x0, void *stream) {
    clear_error();
    int rc = validate_problem(pw);
    if (rc) return rc;
    if (!x0) return fail(STPI_EINVAL, "NULL x0");
    if (shift < 0 || shift > pw->T) return fail(STPI_EINVAL, "shift must be in [0, q]");
    if (shift < pw->T && !x_prev) return fail(STPI_EINVAL, "x_prev is needed when the windows overlap");
    if (x_prev == x0 && shift > 0 && shift < pw->T) return fail(STPI_EINVAL, "x0 must not alias x_prev");
    const size_t plane = (size_t)pw->H * pw->W;
    const double c = 1.0 / std::sqrt((double)plane * pw->T);
    hipStream_t st = (hipStream_t)stream;
    switch (pw->dtype) {
        case STPI_F32:
            hipLaunchKernelGGL(window_start_kernel<float>, dim3(1024), dim3(256), 0, st, (const float *)x_prev,
                               (float *)x0, plane, pw->T, shift, c);
            break;
        case STPI_BF16:
            hipLaunchKernelGGL(window_start_kernel<bf16>, dim3(1024), dim3(256), 0, st, (const bf16 *)x_prev,
                               (bf16 *)x0, plane, pw->T, shift, c);
            break;
        default:
            hipLaunchKernelGGL(window_start_kernel<double>, dim3(1024), dim3(256), 0, st, (const double *)x_prev,
                               (double *)x0, plane, pw->T, shift, c);
    }
    const hipError_t e = hipGetLastError();
    return e == hipSuccess ? STPI_OK : hip_fail(e, "window start launch");
}

}  // extern "C"
