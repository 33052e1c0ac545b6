// The paper's learning objective (SFSeg++) on the single-field operator:
//   - the sigmoid-affine channel combination with bias (Sec. 3, Eq. 9):
//     f = sigmoid(sum_c w_c fc_c + b), and its backward;
//   - soft-binarisation of an iterate (Alg. 1, step 3, with the sigmoid's
//     parameter made explicit): b = sigmoid(kappa (sqrt(N) z / ||z|| - theta)),
//     and its backward through the normalisations around it;
//   - the Focal-Dice loss (Eq. 12) per frame with the soft Dice
//     D_t = (2 sum x gt + eps) / (sum x + sum gt + eps), J = sum_t (1 - D_t)^gamma.
// Reductions: fixed-grid block partials in double, reduced in a fixed order.
#include <hip/hip_runtime.h>

#include <cmath>

#include "../../include/stpi.h"
#include "common.hpp"
#include "host_internal.hpp"

namespace stpi {
namespace {

constexpr int PP_THREADS = 256;
constexpr int PP_BLOCKS = 256;      // grid of the whole-volume reductions
constexpr int FD_BLOCKS = 16;       // blocks per frame in the Focal-Dice sums

__device__ __forceinline__ double sigmoid_d(double a) { return 0.5 * (1.0 + tanh(0.5 * a)); }

template <class ST>
__global__ void combine_sigmoid_fwd_kernel(int C, size_t n, const ST *fc, const double *w, const double *b, ST *f) {
    using CT = typename Compute<ST>::type;
    for (size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (size_t)gridDim.x * blockDim.x) {
        double a = *b;
        for (int c = 0; c < C; ++c) a = fma(w[c], (double)ld(fc + (size_t)c * n + i), a);
        st(f + i, (CT)sigmoid_d(a));
    }
}

// partials[block][c] = sum over the block's elements of g_f f (1 - f) fc_c, c < C;
// partials[block][C] = sum of g_f f (1 - f).
template <class ST>
__global__ void combine_sigmoid_bwd_kernel(int C, size_t n, const ST *fc, const ST *f, const ST *g_f,
                                           double *partials) {
    __shared__ double red[PP_THREADS / 64];
    double acc[STPI_MAX_CHANNELS + 1];
    for (int c = 0; c <= C; ++c) acc[c] = 0.0;
    for (size_t i = (size_t)blockIdx.x * PP_THREADS + threadIdx.x; i < n; i += (size_t)gridDim.x * PP_THREADS) {
        const double fv = (double)ld(f + i);
        const double ga = (double)ld(g_f + i) * fv * (1.0 - fv);
        for (int c = 0; c < C; ++c) acc[c] = fma(ga, (double)ld(fc + (size_t)c * n + i), acc[c]);
        acc[C] += ga;
    }
    for (int c = 0; c <= C; ++c) {
        const double s = block_sum<PP_THREADS>(acc[c], red);
        if (threadIdx.x == 0) partials[(size_t)blockIdx.x * (C + 1) + c] = s;
    }
}

__global__ void combine_sigmoid_bwd_finalize(int C, int nb, const double *partials, double *g_wb) {
    const int c = threadIdx.x;
    if (c > C) return;
    double s = 0.0;
    for (int blk = 0; blk < nb; ++blk) s += partials[(size_t)blk * (C + 1) + c];
    g_wb[c] = s;
}

// b = sigmoid(kappa (sqrt(n) z / ||z|| - theta)); partials of sum b^2.
template <class ST>
__global__ void softbin_fwd_kernel(size_t n, const ST *z, const double *znorm, double kappa, double theta, ST *b,
                                   double *partials) {
    using CT = typename Compute<ST>::type;
    __shared__ double red[PP_THREADS / 64];
    const double sc = sqrt((double)n) / *znorm;
    double acc = 0.0;
    for (size_t i = (size_t)blockIdx.x * PP_THREADS + threadIdx.x; i < n; i += (size_t)gridDim.x * PP_THREADS) {
        const CT v = (CT)sigmoid_d(kappa * ((double)ld(z + i) * sc - theta));
        st(b + i, v);
        const double vs = (double)stored_value(b + i, v);
        acc = fma(vs, vs, acc);
    }
    const double s = block_sum<PP_THREADS>(acc, red);
    if (threadIdx.x == 0) partials[blockIdx.x] = s;
}

__global__ void sqrt_sum_kernel(int nb, const double *partials, double *out) {
    if (threadIdx.x != 0 || blockIdx.x != 0) return;
    double s = 0.0;
    for (int i = 0; i < nb; ++i) s += partials[i];
    *out = sqrt(s);
}

__global__ void sum_kernel(int nb, const double *partials, double *out) {
    if (threadIdx.x != 0 || blockIdx.x != 0) return;
    double s = 0.0;
    for (int i = 0; i < nb; ++i) s += partials[i];
    *out = s;
}

// Backward of b = softbin(y), y = z_prev / ||z_prev||, with g given w.r.t.
// x = b / ||b|| (unit = 1: g_b = (g - x <x, g>) / ||b||, <x, g> = *d) or
// w.r.t. b itself (unit = 0): g_y = g_b b (1 - b) kappa sqrt(n); partials of
// <y, g_y>.
template <class ST>
__global__ void softbin_bwd_kernel(size_t n, int unit, const ST *g, const double *d, const ST *b,
                                   const double *bnorm, const ST *z_prev, const double *znorm_prev, double kappa,
                                   ST *g_y, double *partials) {
    using CT = typename Compute<ST>::type;
    __shared__ double red[PP_THREADS / 64];
    const double ib = unit ? 1.0 / *bnorm : 1.0;
    const double dd = unit ? *d : 0.0;
    const double ks = kappa * sqrt((double)n);
    const double iz = 1.0 / *znorm_prev;
    double acc = 0.0;
    for (size_t i = (size_t)blockIdx.x * PP_THREADS + threadIdx.x; i < n; i += (size_t)gridDim.x * PP_THREADS) {
        const double bv = (double)ld(b + i);
        const double gb = ((double)ld(g + i) - bv * ib * dd) * ib;
        const CT gy = (CT)(gb * bv * (1.0 - bv) * ks);
        st(g_y + i, gy);
        acc = fma((double)ld(z_prev + i) * iz, (double)stored_value(g_y + i, gy), acc);
    }
    const double s = block_sum<PP_THREADS>(acc, red);
    if (threadIdx.x == 0) partials[blockIdx.x] = s;
}

// Per-frame sums: partials[(t FD_BLOCKS + blk) 3 + {0, 1, 2}] = sum x gt, sum x, sum gt.
template <class ST>
__global__ void focal_dice_sums_kernel(size_t plane, const ST *x, const uint8_t *gt, double *partials) {
    __shared__ double red[PP_THREADS / 64];
    const int t = blockIdx.y;
    const ST *xt = x + (size_t)t * plane;
    const uint8_t *gtt = gt + (size_t)t * plane;
    double p = 0.0, sx = 0.0, sy = 0.0;
    for (size_t i = (size_t)blockIdx.x * PP_THREADS + threadIdx.x; i < plane; i += (size_t)gridDim.x * PP_THREADS) {
        const double xv = (double)ld(xt + i), yv = gtt[i] ? 1.0 : 0.0;
        p = fma(xv, yv, p);
        sx += xv;
        sy += yv;
    }
    const double a = block_sum<PP_THREADS>(p, red);
    const double b = block_sum<PP_THREADS>(sx, red);
    const double c = block_sum<PP_THREADS>(sy, red);
    if (threadIdx.x == 0) {
        double *o = partials + ((size_t)t * FD_BLOCKS + blockIdx.x) * 3;
        o[0] = a;
        o[1] = b;
        o[2] = c;
    }
}

// One thread per frame: D_t, the loss term and the gradient coefficients
// dJ/dx_i = A_t gt_i + B_t with A_t = 2 J'_t / den_t, B_t = -J'_t (2 P_t + eps) / den_t^2.
__global__ void focal_dice_frames_kernel(int T, const double *partials, double gamma, double eps, double *coef,
                                         double *terms) {
    const int t = blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= T) return;
    double P = 0.0, X = 0.0, Y = 0.0;
    for (int blk = 0; blk < FD_BLOCKS; ++blk) {
        const double *o = partials + ((size_t)t * FD_BLOCKS + blk) * 3;
        P += o[0];
        X += o[1];
        Y += o[2];
    }
    const double den = X + Y + eps;
    const double D = (2.0 * P + eps) / den;
    const double om = 1.0 - D;
    terms[t] = pow(om, gamma);
    const double dJ = -gamma * pow(om, gamma - 1.0);
    coef[2 * t] = 2.0 * dJ / den;
    coef[2 * t + 1] = -dJ * (2.0 * P + eps) / (den * den);
}

template <class ST>
__global__ void focal_dice_grad_kernel(size_t plane, const uint8_t *gt, const double *coef, ST *g) {
    using CT = typename Compute<ST>::type;
    const int t = blockIdx.y;
    const double A = coef[2 * t], B = coef[2 * t + 1];
    for (size_t i = (size_t)blockIdx.x * PP_THREADS + threadIdx.x; i < plane; i += (size_t)gridDim.x * PP_THREADS)
        st(g + (size_t)t * plane + i, (CT)(gt[(size_t)t * plane + i] ? A + B : B));
}

int pp_check(int64_t n, int dtype) {
    if (n < 1) return fail(STPI_EINVAL, "n must be >= 1");
    if (dtype != STPI_F32 && dtype != STPI_F64) return fail(STPI_EUNSUPPORTED, "float or double volumes only");
    return STPI_OK;
}

}  // namespace
}  // namespace stpi

using namespace stpi;

extern "C" {

int stpi_combine_sigmoid_fwd(int C, int64_t n, int dtype, const void *fc, const double *w, const double *b, void *f,
                             void *stream) {
    clear_error();
    int rc = pp_check(n, dtype);
    if (rc) return rc;
    if (C < 1 || C > STPI_MAX_CHANNELS) return fail(STPI_EINVAL, "C must be in [1, %d]", STPI_MAX_CHANNELS);
    if (!fc || !w || !b || !f) return fail(STPI_EINVAL, "NULL buffer");
    if (f == fc) return fail(STPI_EINVAL, "f must not alias fc");
    hipStream_t st = (hipStream_t)stream;
    if (dtype == STPI_F64)
        hipLaunchKernelGGL(combine_sigmoid_fwd_kernel<double>, dim3(1024), dim3(PP_THREADS), 0, st, C, (size_t)n,
                           (const double *)fc, w, b, (double *)f);
    else
        hipLaunchKernelGGL(combine_sigmoid_fwd_kernel<float>, dim3(1024), dim3(PP_THREADS), 0, st, C, (size_t)n,
                           (const float *)fc, w, b, (float *)f);
    const hipError_t e = hipGetLastError();
    return e == hipSuccess ? STPI_OK : hip_fail(e, "combine sigmoid forward");
}

int stpi_combine_sigmoid_bwd(int C, int64_t n, int dtype, const void *fc, const void *f, const void *g_f,
                             double *g_wb, void *ws, size_t ws_bytes, void *stream) {
    clear_error();
    int rc = pp_check(n, dtype);
    if (rc) return rc;
    if (C < 1 || C > STPI_MAX_CHANNELS) return fail(STPI_EINVAL, "C must be in [1, %d]", STPI_MAX_CHANNELS);
    if (!fc || !f || !g_f || !g_wb) return fail(STPI_EINVAL, "NULL buffer");
    const size_t need = (size_t)PP_BLOCKS * (C + 1) * sizeof(double);
    if (!ws || ws_bytes < need) return fail(STPI_EWORKSPACE, "workspace needs %zu bytes", need);
    hipStream_t st = (hipStream_t)stream;
    double *partials = (double *)ws;
    if (dtype == STPI_F64)
        hipLaunchKernelGGL(combine_sigmoid_bwd_kernel<double>, dim3(PP_BLOCKS), dim3(PP_THREADS), 0, st, C,
                           (size_t)n, (const double *)fc, (const double *)f, (const double *)g_f, partials);
    else
        hipLaunchKernelGGL(combine_sigmoid_bwd_kernel<float>, dim3(PP_BLOCKS), dim3(PP_THREADS), 0, st, C,
                           (size_t)n, (const float *)fc, (const float *)f, (const float *)g_f, partials);
    hipLaunchKernelGGL(combine_sigmoid_bwd_finalize, dim3(1), dim3(128), 0, st, C, PP_BLOCKS, partials, g_wb);
    const hipError_t e = hipGetLastError();
    return e == hipSuccess ? STPI_OK : hip_fail(e, "combine sigmoid backward");
}

int stpi_softbin_fwd(int64_t n, int dtype, const void *z, const double *znorm, double kappa, double theta, void *b,
                     double *bnorm, void *ws, size_t ws_bytes, void *stream) {
    clear_error();
    int rc = pp_check(n, dtype);
    if (rc) return rc;
    if (!z || !znorm || !b || !bnorm) return fail(STPI_EINVAL, "NULL buffer");
    if (b == z) return fail(STPI_EINVAL, "b must not alias z");
    if (!std::isfinite(kappa) || !std::isfinite(theta)) return fail(STPI_EINVAL, "kappa and theta must be finite");
    if (!ws || ws_bytes < (size_t)PP_BLOCKS * sizeof(double))
        return fail(STPI_EWORKSPACE, "workspace needs %zu bytes", (size_t)PP_BLOCKS * sizeof(double));
    hipStream_t st = (hipStream_t)stream;
    double *partials = (double *)ws;
    if (dtype == STPI_F64)
        hipLaunchKernelGGL(softbin_fwd_kernel<double>, dim3(PP_BLOCKS), dim3(PP_THREADS), 0, st, (size_t)n,
                           (const double *)z, znorm, kappa, theta, (double *)b, partials);
    else
        hipLaunchKernelGGL(softbin_fwd_kernel<float>, dim3(PP_BLOCKS), dim3(PP_THREADS), 0, st, (size_t)n,
                           (const float *)z, znorm, kappa, theta, (float *)b, partials);
    hipLaunchKernelGGL(sqrt_sum_kernel, dim3(1), dim3(64), 0, st, PP_BLOCKS, partials, bnorm);
    const hipError_t e = hipGetLastError();
    return e == hipSuccess ? STPI_OK : hip_fail(e, "softbin forward");
}

int stpi_softbin_bwd(int64_t n, int dtype, int unit, const void *g, const double *d, const void *b,
                     const double *bnorm, const void *z_prev, const double *znorm_prev, double kappa, void *g_y,
                     double *d_prev, void *ws, size_t ws_bytes, void *stream) {
    clear_error();
    int rc = pp_check(n, dtype);
    if (rc) return rc;
    if (!g || !b || !z_prev || !znorm_prev || !g_y || !d_prev || (unit && (!d || !bnorm)))
        return fail(STPI_EINVAL, "NULL buffer");
    if (g_y == g || g_y == b || g_y == z_prev) return fail(STPI_EINVAL, "g_y must not alias an input");
    if (!std::isfinite(kappa)) return fail(STPI_EINVAL, "kappa must be finite");
    if (!ws || ws_bytes < (size_t)PP_BLOCKS * sizeof(double))
        return fail(STPI_EWORKSPACE, "workspace needs %zu bytes", (size_t)PP_BLOCKS * sizeof(double));
    hipStream_t st = (hipStream_t)stream;
    double *partials = (double *)ws;
    if (dtype == STPI_F64)
        hipLaunchKernelGGL(softbin_bwd_kernel<double>, dim3(PP_BLOCKS), dim3(PP_THREADS), 0, st, (size_t)n, unit,
                           (const double *)g, d, (const double *)b, bnorm, (const double *)z_prev, znorm_prev, kappa,
                           (double *)g_y, partials);
    else
        hipLaunchKernelGGL(softbin_bwd_kernel<float>, dim3(PP_BLOCKS), dim3(PP_THREADS), 0, st, (size_t)n, unit,
                           (const float *)g, d, (const float *)b, bnorm, (const float *)z_prev, znorm_prev, kappa,
                           (float *)g_y, partials);
    hipLaunchKernelGGL(sum_kernel, dim3(1), dim3(64), 0, st, PP_BLOCKS, partials, d_prev);
    const hipError_t e = hipGetLastError();
    return e == hipSuccess ? STPI_OK : hip_fail(e, "softbin backward");
}

size_t stpi_focal_dice_workspace_bytes(int T) {
    return T < 1 ? 0 : (size_t)T * (3 * FD_BLOCKS + 2 + 1) * sizeof(double);
}

int stpi_focal_dice(int T, int64_t plane, int dtype, const void *x, const uint8_t *gt, double gamma, double eps,
                    double *loss, void *g_x, void *ws, size_t ws_bytes, void *stream) {
    clear_error();
    if (T < 1 || plane < 1) return fail(STPI_EINVAL, "empty volume");
    int rc = pp_check(plane, dtype);
    if (rc) return rc;
    if (!x || !gt || !loss || !g_x) return fail(STPI_EINVAL, "NULL buffer");
    if (g_x == x) return fail(STPI_EINVAL, "g_x must not alias x");
    if (!(gamma > 0.0) || !std::isfinite(gamma) || !(eps > 0.0) || !std::isfinite(eps))
        return fail(STPI_EINVAL, "gamma and eps must be finite and > 0");
    const size_t need = stpi_focal_dice_workspace_bytes(T);
    if (!ws || ws_bytes < need) return fail(STPI_EWORKSPACE, "workspace needs %zu bytes", need);
    hipStream_t st = (hipStream_t)stream;
    double *partials = (double *)ws;
    double *coef = partials + (size_t)T * 3 * FD_BLOCKS;
    double *terms = coef + 2 * (size_t)T;
    if (dtype == STPI_F64)
        hipLaunchKernelGGL(focal_dice_sums_kernel<double>, dim3(FD_BLOCKS, T), dim3(PP_THREADS), 0, st,
                           (size_t)plane, (const double *)x, gt, partials);
    else
        hipLaunchKernelGGL(focal_dice_sums_kernel<float>, dim3(FD_BLOCKS, T), dim3(PP_THREADS), 0, st,
                           (size_t)plane, (const float *)x, gt, partials);
    hipLaunchKernelGGL(focal_dice_frames_kernel, dim3((T + 63) / 64), dim3(64), 0, st, T, partials, gamma, eps, coef,
                       terms);
    hipLaunchKernelGGL(sum_kernel, dim3(1), dim3(64), 0, st, T, terms, loss);
    if (dtype == STPI_F64)
        hipLaunchKernelGGL(focal_dice_grad_kernel<double>, dim3(64, T), dim3(PP_THREADS), 0, st, (size_t)plane, gt,
                           coef, (double *)g_x);
    else
        hipLaunchKernelGGL(focal_dice_grad_kernel<float>, dim3(64, T), dim3(PP_THREADS), 0, st, (size_t)plane, gt,
                           coef, (float *)g_x);
    const hipError_t e = hipGetLastError();
    return e == hipSuccess ? STPI_OK : hip_fail(e, "focal dice");
}

}  // extern "C"
