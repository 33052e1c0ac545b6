// Full SFSeg operator (Eq. 7 with alpha > 0 and a unary map distinct from the
// pairwise feature): kernel instantiations and the C ABI.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstring>

#include "../../include/stpi.h"
#include "chain.hpp"
#include "host_internal.hpp"
#include "sfseg.hpp"

namespace stpi {
namespace {

#define STPI_SFSEG_ENTRY(ST, RS, RT, TH, TW, NTHR, RY, QX) \
    {RS, RT, TH, TW, NTHR, &launch_sfseg<ST, RS, RT, TH, TW, NTHR, RY, QX>, &sfseg_blocks_per_cu<ST, RS, RT, TH, TW, NTHR, RY, QX>}

// Compiled (RS, RT) pairs: the smallest one covering the problem's radii is used.
const SfsegVariant kSfsegF32[] = {
    STPI_SFSEG_ENTRY(float, 4, 2, 16, 64, 256, 8, 4),
    STPI_SFSEG_ENTRY(float, 8, 3, 16, 64, 256, 8, 4),
    STPI_SFSEG_ENTRY(float, 16, 5, 32, 64, 512, 8, 4),
};
const SfsegVariant kSfsegF64[] = {
    STPI_SFSEG_ENTRY(double, 4, 2, 16, 64, 256, 8, 4),
};

const SfsegVariant *sfseg_variant(const stpi_problem *p) {
    const SfsegVariant *list = p->dtype == STPI_F64 ? kSfsegF64 : kSfsegF32;
    const int n = p->dtype == STPI_F64 ? (int)(sizeof(kSfsegF64) / sizeof(kSfsegF64[0]))
                                       : (int)(sizeof(kSfsegF32) / sizeof(kSfsegF32[0]));
    for (int i = 0; i < n; ++i)
        if (list[i].RS >= p->r_s && list[i].RT >= p->r_t) return &list[i];
    return nullptr;
}

int sfseg_tiles(const SfsegVariant &v, const stpi_problem *p) {
    return ((p->W + v.TW - 1) / v.TW) * ((p->H + v.TH - 1) / v.TH);
}

// Frame segments per tile: enough work units to fill the resident slots when
// the frame has few tiles, each segment at least 4 r_t frames long; a tile
// left whole is split as the single-field step splits it (split_short_tiles).
int sfseg_segments(const SfsegVariant &v, const stpi_problem *p) {
    const int tiles = sfseg_tiles(v, p);
    const int resident = device_cus() * v.blocks_per_cu();
    const int rt = std::max(v.RT, 1);
    int nseg = std::min(std::min(resident / std::max(tiles, 1), p->T / (4 * rt)), STPI_NSEG_MAX);
    if (nseg < 1) nseg = 1;
    if (nseg == 1) nseg = split_short_tiles(std::max(tiles, 1), p->T, v.RT);
    return nseg;
}

struct SfsegLayout {
    size_t partials_off, partials_cap, buf_off, total;
};

SfsegLayout sfseg_layout(const stpi_problem *p, const SfsegVariant &v) {
    SfsegLayout L;
    const size_t elem = p->dtype == STPI_F64 ? 8 : 4;
    L.partials_off = 256;
    L.partials_cap = std::max((size_t)sfseg_tiles(v, p) * STPI_NSEG_MAX, (size_t)std::max(NORM_BLOCKS_HOST,
                                                                                        SFSEG_RANGE_BLOCKS));
    size_t off = L.partials_off + ((L.partials_cap * 3 * sizeof(double) + 255) & ~(size_t)255);
    L.buf_off = off;
    L.total = off + (((size_t)p->T * p->H * p->W * elem + 255) & ~(size_t)255);
    return L;
}

int sfseg_check(const stpi_problem *p, const SfsegVariant **v) {
    int rc = validate_problem(p);
    if (rc) return rc;
    if (p->dtype != STPI_F32 && p->dtype != STPI_F64) return fail(STPI_EUNSUPPORTED, "sfseg: float or double only");
    *v = sfseg_variant(p);
    if (!*v) return fail(STPI_EUNSUPPORTED, "sfseg: no compiled kernel for radii (%d, %d)", p->r_s, p->r_t);
    return STPI_OK;
}

void sfseg_fill(SfsegLaunch &L, const stpi_problem *p, const void *s, const void *f, double alpha) {
    std::memset(&L, 0, sizeof(L));
    L.s = s;
    L.f = f;
    L.ainv = 1.0 / alpha;
    L.T = p->T;
    L.H = p->H;
    L.W = p->W;
    make_taps(p, L.gs, L.gt);
}

// states: flags |= FLAG_AFFINITY and done when some affinity of Eq. 2 can be
// negative (alpha (max f - min f)^2 > 1, a negative s, or a NaN).
__global__ void sfseg_range_check_kernel(const double *partials, int n, double alpha, DevState *s) {
    if (threadIdx.x != 0 || blockIdx.x != 0) return;
    double fmn = INFINITY, fmx = -INFINITY, smn = INFINITY;
    bool nan = false;
    for (int b = 0; b < n; ++b) {
        const double a = partials[3 * b], c = partials[3 * b + 1], e = partials[3 * b + 2];
        nan |= a != a || c != c || e != e;
        fmn = fmin(fmn, a);
        fmx = fmax(fmx, c);
        smn = fmin(smn, e);
    }
    const double d = fmx - fmn;
    if (nan || smn < 0.0 || alpha * d * d > 1.0) {
        s->flags |= FLAG_AFFINITY;
        s->done = 1;
    }
}

template <class ST>
hipError_t sfseg_range(size_t n, const void *s, const void *f, double *partials, double alpha, DevState *state,
                       hipStream_t st) {
    hipLaunchKernelGGL(sfseg_range_kernel<ST>, dim3(SFSEG_RANGE_BLOCKS), dim3(256), 0, st, n, (const ST *)s,
                       (const ST *)f, partials);
    hipLaunchKernelGGL(sfseg_range_check_kernel, dim3(1), dim3(64), 0, st, partials, SFSEG_RANGE_BLOCKS, alpha,
                       state);
    return hipGetLastError();
}

}  // namespace
}  // namespace stpi

using namespace stpi;

extern "C" {

int stpi_sfseg_unary(int64_t n, int dtype, const void *S, double p, void *s, void *stream) {
    clear_error();
    if (n < 1 || !S || !s) return fail(STPI_EINVAL, "sfseg_unary: empty volume or NULL buffer");
    if (!std::isfinite(p) || p < 0.0) return fail(STPI_EINVAL, "sfseg_unary: p must be finite and >= 0");
    hipStream_t st = (hipStream_t)stream;
    if (dtype == STPI_F32)
        hipLaunchKernelGGL(sfseg_unary_kernel<float>, dim3(1024), dim3(256), 0, st, (size_t)n, (const float *)S, p,
                           (float *)s);
    else if (dtype == STPI_F64)
        hipLaunchKernelGGL(sfseg_unary_kernel<double>, dim3(1024), dim3(256), 0, st, (size_t)n, (const double *)S,
                           p, (double *)s);
    else
        return fail(STPI_EUNSUPPORTED, "sfseg_unary: float or double only");
    const hipError_t e = hipGetLastError();
    return e == hipSuccess ? STPI_OK : hip_fail(e, "sfseg_unary launch");
}

size_t stpi_sfseg_workspace_bytes(const stpi_problem *p) {
    const SfsegVariant *v = nullptr;
    if (sfseg_check(p, &v) != STPI_OK) return 0;
    return sfseg_layout(p, *v).total;
}

int stpi_sfseg_step(const stpi_problem *p, const void *s, const void *f, double alpha, const void *x,
                    double x_scale, void *z, double *d_sums, void *ws, size_t ws_bytes, void *stream) {
    clear_error();
    const SfsegVariant *v = nullptr;
    int rc = sfseg_check(p, &v);
    if (rc) return rc;
    if (!s || !f || !x || !z || !d_sums) return fail(STPI_EINVAL, "NULL buffer");
    if (z == s || z == f || z == x) return fail(STPI_EINVAL, "z must not alias s, f or x");
    if (!(alpha > 0.0) || !std::isfinite(alpha)) return fail(STPI_EINVAL, "alpha must be finite and > 0");
    if (!std::isfinite(x_scale)) return fail(STPI_EINVAL, "x_scale must be finite");
    const SfsegLayout L = sfseg_layout(p, *v);
    if (!ws || ws_bytes < L.total) return fail(STPI_EWORKSPACE, "sfseg workspace needs %zu bytes", L.total);
    hipStream_t st = (hipStream_t)stream;
    SfsegLaunch SL;
    sfseg_fill(SL, p, s, f, alpha);
    SL.buf0 = const_cast<void *>(x);
    SL.buf1 = z;
    SL.x_scale = x_scale;
    SL.partials = (double *)((char *)ws + L.partials_off);
    SL.nseg = sfseg_segments(*v, p);
    hipError_t e = v->launch(SL, st);
    if (e != hipSuccess) return hip_fail(e, "sfseg step launch");
    e = launch_step_sums(SL.partials, sfseg_tiles(*v, p) * SL.nseg, x_scale, d_sums, st);
    return e == hipSuccess ? STPI_OK : hip_fail(e, "step sums launch");
}

int stpi_sfseg_iterate(const stpi_problem *p, const void *s, const void *f, double alpha, void *x, int init,
                       int max_iters, double tol, void *ws, size_t ws_bytes, stpi_result *out, void *stream) {
    clear_error();
    const SfsegVariant *v = nullptr;
    int rc = sfseg_check(p, &v);
    if (rc) return rc;
    if (!s || !f || !x || !out) return fail(STPI_EINVAL, "NULL buffer or result");
    if (x == s || x == f) return fail(STPI_EINVAL, "x must not alias s or f");
    if (!(alpha > 0.0) || !std::isfinite(alpha)) return fail(STPI_EINVAL, "alpha must be finite and > 0");
    if (max_iters < 0) return fail(STPI_EINVAL, "max_iters must be >= 0");
    if (init != 0 && init != 1) return fail(STPI_EINVAL, "init must be 0 (use x) or 1 (uniform)");
    if (!std::isfinite(tol)) return fail(STPI_EINVAL, "tol must be finite");
    const SfsegLayout L = sfseg_layout(p, *v);
    if (!ws || ws_bytes < L.total) return fail(STPI_EWORKSPACE, "sfseg workspace needs %zu bytes", L.total);
    std::memset(out, 0, sizeof(*out));
    hipStream_t st = (hipStream_t)stream;
    const DtypeOps *ops = ops_for(p->dtype);
    const size_t N = (size_t)p->T * p->H * p->W;
    DevState *state = (DevState *)ws;
    double *partials = (double *)((char *)ws + L.partials_off);
    void *buf1 = (char *)ws + L.buf_off;
    hipError_t e;
    // start vector and state (as stpi_iterate's plain form)
    if (init == 1) {
        if ((e = ops->fill_ones(x, N, st)) != hipSuccess) return hip_fail(e, "fill");
        if ((e = launch_state_init(state, 1.0 / std::sqrt((double)N), tol, max_iters, 0, 0, st)) != hipSuccess)
            return hip_fail(e, "init");
    } else {
        if ((e = launch_state_init(state, 1.0, tol, max_iters, 0, 0, st)) != hipSuccess) return hip_fail(e, "init");
        if ((e = ops->sumsq(x, N, partials, st)) != hipSuccess) return hip_fail(e, "norm");
        if ((e = launch_state_from_norm(partials, NORM_BLOCKS_HOST, state, st)) != hipSuccess)
            return hip_fail(e, "init norm");
    }
    e = p->dtype == STPI_F64 ? sfseg_range<double>(N, s, f, partials, alpha, state, st)
                             : sfseg_range<float>(N, s, f, partials, alpha, state, st);
    if (e != hipSuccess) return hip_fail(e, "affinity range check");
    SfsegLaunch SL;
    sfseg_fill(SL, p, s, f, alpha);
    SL.buf0 = x;
    SL.buf1 = buf1;
    SL.state = state;
    SL.partials = partials;
    SL.nseg = sfseg_segments(*v, p);
    SL.fuse = v->NTHR >= FINAL_THREADS && !fusion_disabled() ? 1 : 0;
    const int nunits = sfseg_tiles(*v, p) * SL.nseg;
    if ((e = launch_partials_empty(partials, nunits, st)) != hipSuccess) return hip_fail(e, "partials");
    // steps in chunks; a tolerance run checks the stop flag after each chunk
    DevState hs;
    for (int done = 0; done < max_iters;) {
        const int n = tol > 0.0 ? std::min(CHAIN_CHUNK, max_iters - done) : max_iters;
        for (int k = 0; k < n; ++k) {
            if ((e = v->launch(SL, st)) != hipSuccess) return hip_fail(e, "sfseg step launch");
            if (!SL.fuse && (e = launch_finalize(partials, nunits, state, st)) != hipSuccess)
                return hip_fail(e, "finalize launch");
        }
        done += n;
        if (done < max_iters) {
            if ((e = hipMemcpyAsync(&hs, state, sizeof(hs), hipMemcpyDeviceToHost, st)) != hipSuccess ||
                (e = hipStreamSynchronize(st)) != hipSuccess)
                return hip_fail(e, "stop check");
            if (hs.done) break;
        }
    }
    if ((e = ops->normalize(x, buf1, N, state, st)) != hipSuccess) return hip_fail(e, "normalize");
    if ((e = hipMemcpyAsync(&hs, state, sizeof(hs), hipMemcpyDeviceToHost, st)) != hipSuccess ||
        (e = hipStreamSynchronize(st)) != hipSuccess)
        return hip_fail(e, "state readback");
    out->iters = hs.iters;
    out->converged = hs.converged;
    out->flags = hs.flags;
    out->residual = hs.residual;
    out->lambda = hs.lambda;
    out->rayleigh = hs.rayleigh;
    out->first_residuals[0] = hs.first_res[0];
    out->first_residuals[1] = hs.first_res[1];
    if (hs.flags & FLAG_AFFINITY) {
        out->status = STPI_EINVAL;
        return fail(STPI_EINVAL, "sfseg: an affinity 1 - alpha (f_i - f_j)^2 can be negative (alpha (max f - min f)^2 "
                                 "> 1), or s has a negative or NaN value");
    }
    if (hs.flags & FLAG_SYNC) {
        out->status = STPI_EHIP;
        return fail(STPI_EHIP, "a step's partial sums did not arrive (step %d)", hs.iters + 1);
    }
    out->status = (hs.flags & FLAG_NONFINITE) ? STPI_ENONFINITE : (hs.flags & FLAG_ZERO) ? STPI_EZERO_NORM : 0;
    if (out->status) return fail(out->status, "iteration stopped after %d steps: %s", hs.iters,
                                 stpi_status_string(out->status));
    return STPI_OK;
}

}  // extern "C"
