// Grid transfer for the two-level start: box-average restriction of a volume
// to a coarse grid and its prolongation back (nearest cell or cell-centred
// trilinear), optionally multiplied by a fine field. One thread per output
// voxel; arithmetic in float (double for double storage).
#include <hip/hip_runtime.h>

#include <algorithm>

#include "../../include/stpi.h"
#include "common.hpp"
#include "host_internal.hpp"

namespace stpi {

struct CoarseDims {
    int T, H, W;     // fine
    int Tc, Hc, Wc;  // coarse: ceil(T / st), ceil(H / sy), ceil(W / sy)
    int sy, st;
};

template <class ST>
__global__ void downsample_kernel(CoarseDims d, const ST *in, ST *out) {
    using CT = typename Compute<ST>::type;
    const size_t nc = (size_t)d.Tc * d.Hc * d.Wc;
    for (size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x; i < nc; i += (size_t)gridDim.x * blockDim.x) {
        const int xc = (int)(i % d.Wc);
        const int yc = (int)((i / d.Wc) % d.Hc);
        const int tc = (int)(i / ((size_t)d.Wc * d.Hc));
        const int t1 = min(d.T, (tc + 1) * d.st), y1 = min(d.H, (yc + 1) * d.sy), x1 = min(d.W, (xc + 1) * d.sy);
        CT s = CT(0);
        int cnt = 0;
        for (int t = tc * d.st; t < t1; ++t)
            for (int y = yc * d.sy; y < y1; ++y) {
                const ST *row = in + ((size_t)t * d.H + y) * d.W;
                for (int x = xc * d.sy; x < x1; ++x) {
                    s += ld(row + x);
                    ++cnt;
                }
            }
        st(out + i, s / CT(cnt));
    }
}

// Cell-centred linear coordinate of fine index i on an axis of coarse size n
// and scale s: c = (i + 1/2) / s - 1/2, clamped to [0, n - 1].
template <class CT>
__device__ __forceinline__ void lin_axis(int i, int s, int n, int &i0, int &i1, CT &w) {
    CT c = (CT(i) + CT(0.5)) / CT(s) - CT(0.5);
    c = c < CT(0) ? CT(0) : (c > CT(n - 1) ? CT(n - 1) : c);
    i0 = (int)c;
    i1 = i0 + 1 < n ? i0 + 1 : n - 1;
    w = c - CT(i0);
}

template <class ST>
__global__ void upsample_kernel(CoarseDims d, int mode, const ST *in, const ST *mul, ST *out) {
    using CT = typename Compute<ST>::type;
    const size_t n = (size_t)d.T * d.H * d.W;
    for (size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (size_t)gridDim.x * blockDim.x) {
        const int x = (int)(i % d.W);
        const int y = (int)((i / d.W) % d.H);
        const int t = (int)(i / ((size_t)d.W * d.H));
        CT v;
        if (mode == 0) {
            v = ld(in + ((size_t)(t / d.st) * d.Hc + y / d.sy) * d.Wc + x / d.sy);
        } else {
            int t0, t1, y0, y1, x0, x1;
            CT wt, wy, wx;
            lin_axis<CT>(t, d.st, d.Tc, t0, t1, wt);
            lin_axis<CT>(y, d.sy, d.Hc, y0, y1, wy);
            lin_axis<CT>(x, d.sy, d.Wc, x0, x1, wx);
            auto at = [&](int tt, int yy, int xx) { return (CT)ld(in + ((size_t)tt * d.Hc + yy) * d.Wc + xx); };
            const CT a0 = at(t0, y0, x0) + wx * (at(t0, y0, x1) - at(t0, y0, x0));
            const CT a1 = at(t0, y1, x0) + wx * (at(t0, y1, x1) - at(t0, y1, x0));
            const CT b0 = at(t1, y0, x0) + wx * (at(t1, y0, x1) - at(t1, y0, x0));
            const CT b1 = at(t1, y1, x0) + wx * (at(t1, y1, x1) - at(t1, y1, x0));
            const CT a = a0 + wy * (a1 - a0), b = b0 + wy * (b1 - b0);
            v = a + wt * (b - a);
        }
        if (mul) v *= (CT)ld(mul + i);
        st(out + i, v);
    }
}

template <class ST>
static hipError_t launch_down(const CoarseDims &d, const void *in, void *out, hipStream_t s) {
    const size_t nc = (size_t)d.Tc * d.Hc * d.Wc;
    const int blocks = (int)std::min<size_t>((nc + 255) / 256, 4096);
    hipLaunchKernelGGL(downsample_kernel<ST>, dim3(blocks), dim3(256), 0, s, d, (const ST *)in, (ST *)out);
    return hipGetLastError();
}

template <class ST>
static hipError_t launch_up(const CoarseDims &d, int mode, const void *in, const void *mul, void *out,
                            hipStream_t s) {
    const size_t n = (size_t)d.T * d.H * d.W;
    const int blocks = (int)std::min<size_t>((n + 255) / 256, 8192);
    hipLaunchKernelGGL(upsample_kernel<ST>, dim3(blocks), dim3(256), 0, s, d, mode, (const ST *)in, (const ST *)mul,
                       (ST *)out);
    return hipGetLastError();
}

// y[i] = x[i] * s (times *s_dev when given), formed in double and rounded to
// the storage type once.
template <class ST>
__global__ void scale_kernel(size_t n, const ST *x, double s, const double *s_dev, ST *y) {
    const double m = s_dev ? s * *s_dev : s;
    for (size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (size_t)gridDim.x * blockDim.x)
        st(y + i, (typename Compute<ST>::type)((double)ld(x + i) * m));
}

template <class ST>
hipError_t launch_scale(size_t n, const void *x, double s, const double *s_dev, void *y, hipStream_t st_) {
    const int blocks = (int)std::min<size_t>((n + 255) / 256, 4096);
    hipLaunchKernelGGL(scale_kernel<ST>, dim3(blocks), dim3(256), 0, st_, n, (const ST *)x, s, s_dev, (ST *)y);
    return hipGetLastError();
}

static int coarse_dims(int T, int H, int W, int sy, int st, int dtype, CoarseDims &d) {
    if (T < 1 || H < 1 || W < 1) return fail(STPI_EINVAL, "volume must be at least 1x1x1 (got %dx%dx%d)", T, H, W);
    if (sy < 1 || st < 1) return fail(STPI_EINVAL, "factors must be >= 1 (got sy %d, st %d)", sy, st);
    if (dtype != STPI_F32 && dtype != STPI_BF16 && dtype != STPI_F64) return fail(STPI_EINVAL, "unknown dtype %d", dtype);
    d.T = T;
    d.H = H;
    d.W = W;
    d.sy = sy;
    d.st = st;
    d.Tc = (T + st - 1) / st;
    d.Hc = (H + sy - 1) / sy;
    d.Wc = (W + sy - 1) / sy;
    return STPI_OK;
}

}  // namespace stpi

using namespace stpi;

extern "C" {

int stpi_downsample(int T, int H, int W, int sy, int st, int dtype, const void *in, void *out, void *stream) {
    clear_error();
    CoarseDims d;
    int rc = coarse_dims(T, H, W, sy, st, dtype, d);
    if (rc) return rc;
    if (!in || !out) return fail(STPI_EINVAL, "NULL buffer");
    if (in == out) return fail(STPI_EINVAL, "out must not alias in");
    hipStream_t s = (hipStream_t)stream;
    hipError_t e = dtype == STPI_F32    ? launch_down<float>(d, in, out, s)
                   : dtype == STPI_BF16 ? launch_down<bf16>(d, in, out, s)
                                        : launch_down<double>(d, in, out, s);
    return e == hipSuccess ? STPI_OK : hip_fail(e, "downsample");
}

int stpi_upsample(int T, int H, int W, int sy, int st, int mode, int dtype, const void *in, const void *mul, void *out,
                  void *stream) {
    clear_error();
    CoarseDims d;
    int rc = coarse_dims(T, H, W, sy, st, dtype, d);
    if (rc) return rc;
    if (mode != 0 && mode != 1) return fail(STPI_EINVAL, "mode must be 0 (nearest) or 1 (linear)");
    if (!in || !out) return fail(STPI_EINVAL, "NULL buffer");
    if (in == out || mul == out) return fail(STPI_EINVAL, "out must not alias in or mul");
    hipStream_t s = (hipStream_t)stream;
    hipError_t e = dtype == STPI_F32    ? launch_up<float>(d, mode, in, mul, out, s)
                   : dtype == STPI_BF16 ? launch_up<bf16>(d, mode, in, mul, out, s)
                                        : launch_up<double>(d, mode, in, mul, out, s);
    return e == hipSuccess ? STPI_OK : hip_fail(e, "upsample");
}

int stpi_coarse_problem(const stpi_problem *fine, int sy, int st, stpi_problem *coarse) {
    clear_error();
    if (!fine || !coarse) return fail(STPI_EINVAL, "NULL problem");
    CoarseDims d;
    int rc = coarse_dims(fine->T, fine->H, fine->W, sy, st, fine->dtype, d);
    if (rc) return rc;
    if (fine->r_s < 0 || fine->r_t < 0 || !(fine->sigma_s > 0.f) || !(fine->sigma_t > 0.f))
        return fail(STPI_EINVAL, "kernel needs sigmas > 0 and radii >= 0");
    stpi_problem c = *fine;
    c.T = d.Tc;
    c.H = d.Hc;
    c.W = d.Wc;
    c.sigma_s = (float)((double)fine->sigma_s / sy);
    c.sigma_t = (float)((double)fine->sigma_t / st);
    c.r_s = (fine->r_s + sy - 1) / sy;
    c.r_t = (fine->r_t + st - 1) / st;
    *coarse = c;
    return STPI_OK;
}

int stpi_scale(int64_t n, int dtype, const void *x, double s, const double *s_dev, void *y, void *stream) {
    clear_error();
    if (n < 0) return fail(STPI_EINVAL, "negative length");
    if (dtype != STPI_F32 && dtype != STPI_BF16 && dtype != STPI_F64) return fail(STPI_EINVAL, "unknown dtype %d", dtype);
    if (n == 0) return STPI_OK;
    if (!x || !y) return fail(STPI_EINVAL, "NULL buffer");
    hipStream_t sm = (hipStream_t)stream;
    hipError_t e = dtype == STPI_F32    ? launch_scale<float>((size_t)n, x, s, s_dev, y, sm)
                   : dtype == STPI_BF16 ? launch_scale<bf16>((size_t)n, x, s, s_dev, y, sm)
                                        : launch_scale<double>((size_t)n, x, s, s_dev, y, sm);
    return e == hipSuccess ? STPI_OK : hip_fail(e, "scale");
}

}  // extern "C"
