// The exact pairwise affinity of Sec. 3, Eq. 1 (before the first-order Taylor
// approximation), applied matrix-free for the comparison of the approximate
// and exact eigenvectors (Sec. 4, "Quantitative analysis"):
//
//   z_i = s_i sum_{j in N(i)} s_j exp(-alpha (f_i - f_j)^2) G_ij x_j.
//
// The weight depends on both endpoints' features, so the filter is not
// separable: each output gathers its whole (2 r_t + 1)(2 r_s + 1)^2 box. A
// workgroup owns a 16 x 16 output tile of one frame; it stages s x and f on
// the halo-extended tile of the 2 r_t + 1 frames around it in LDS (raw buffer
// loads, out-of-range offsets read 0: the zero padding) and each thread sums
// its output's box from LDS. Radii up to (8, 4). Per-workgroup partial sums
// (sum z^2, sum z x_stored) go to a fixed-order reduction, as for the step.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstring>

#include "../../include/stpi.h"
#include "chain.hpp"
#include "host_internal.hpp"
#include "stencil.hpp"

namespace stpi {
namespace {

constexpr int EXP_TILE = 16;
constexpr int EXP_RS = 8, EXP_RT = 4;
constexpr int EXP_HT = EXP_TILE + 2 * EXP_RS;  // halo tile side
constexpr int EXP_THREADS = EXP_TILE * EXP_TILE;

template <class ST>
struct ExpArgs {
    using CT = typename Compute<ST>::type;
    const ST *s, *f;
    ST *buf0, *buf1;
    DevState *state;
    double *partials;
    double x_scale;
    CT alpha;
    int T, H, W, rs, rt;
    CT gs[2 * EXP_RS + 1], gt[2 * EXP_RT + 1];
};

template <class ST>
__global__ __launch_bounds__(EXP_THREADS) void exp_step_kernel(ExpArgs<ST> a) {
    using CT = typename Compute<ST>::type;
    using IO = BufIO<ST>;
    __shared__ CT lu[2 * EXP_RT + 1][EXP_HT * EXP_HT];
    __shared__ CT lf[2 * EXP_RT + 1][EXP_HT * EXP_HT];
    __shared__ double red[EXP_THREADS / 64];
    const int nbx = (a.W + EXP_TILE - 1) / EXP_TILE, nby = (a.H + EXP_TILE - 1) / EXP_TILE;
    const int unit = blockIdx.x;  // (frame, tile)
    const int t = unit / (nbx * nby), tile = unit % (nbx * nby);
    const int x0 = (tile % nbx) * EXP_TILE, y0 = (tile / nbx) * EXP_TILE;
    const ST *src;
    ST *dst;
    double scale;
    if (a.state) {
        if (a.state->done) return;
        const int cur = a.state->cur;
        src = cur ? a.buf1 : a.buf0;
        dst = cur ? a.buf0 : a.buf1;
        scale = a.state->scale;
    } else {
        src = a.buf0;
        dst = a.buf1;
        scale = a.x_scale;
    }
    const size_t plane = (size_t)a.H * a.W;
    const uint32_t pbytes = (uint32_t)(plane * IO::SZ);
    const int tid = threadIdx.x;
    // stage s x scale and f of frames t - rt .. t + rt on the halo tile
    for (int dt = -a.rt; dt <= a.rt; ++dt) {
        const int tt = t + dt;
        const bool fin = tt >= 0 && tt < a.T;
        const size_t fo = fin ? (size_t)tt * plane : 0;
        const auto rs_ = make_rsrc(a.s + fo, fin ? pbytes : 0u);
        const auto rf_ = make_rsrc(a.f + fo, fin ? pbytes : 0u);
        const auto rx_ = make_rsrc(src + fo, fin ? pbytes : 0u);
        for (int e = tid; e < EXP_HT * EXP_HT; e += EXP_THREADS) {
            const int gy = y0 - EXP_RS + e / EXP_HT, gx = x0 - EXP_RS + e % EXP_HT;
            const uint32_t off =
                ((unsigned)gy < (unsigned)a.H && (unsigned)gx < (unsigned)a.W) ? (uint32_t)(gy * a.W + gx) * IO::SZ
                                                                                : OOB;
            lu[dt + EXP_RT][e] = IO::load(rs_, off) * IO::load(rx_, off) * (CT)scale;
            lf[dt + EXP_RT][e] = IO::load(rf_, off);
        }
    }
    __syncthreads();
    const int ly = tid / EXP_TILE, lx = tid % EXP_TILE;
    const int gy = y0 + ly, gx = x0 + lx;
    double d1 = 0.0, d2 = 0.0;
    if (gy < a.H && gx < a.W) {
        const int c = (ly + EXP_RS) * EXP_HT + lx + EXP_RS;
        const CT fi = lf[EXP_RT][c];
        CT acc = CT(0);
        for (int dt = -a.rt; dt <= a.rt; ++dt) {
            const CT wt = a.gt[dt + EXP_RT];
            for (int dy = -a.rs; dy <= a.rs; ++dy) {
                const CT wty = wt * a.gs[dy + EXP_RS];
                const CT *ur = &lu[dt + EXP_RT][c + dy * EXP_HT];
                const CT *fr = &lf[dt + EXP_RT][c + dy * EXP_HT];
                for (int dx = -a.rs; dx <= a.rs; ++dx) {
                    const CT d = fi - fr[dx];
                    acc = fma(wty * a.gs[dx + EXP_RS] * exp(-a.alpha * d * d), ur[dx], acc);
                }
            }
        }
        const size_t i = (size_t)t * plane + (size_t)gy * a.W + gx;
        const CT z = ld(a.s + i) * acc;
        st(dst + i, z);
        const double zs = (double)stored_value(dst + i, z);
        d2 = zs * zs;
        d1 = zs * (double)ld(src + i);
    }
    const double s1 = block_sum<EXP_THREADS>(d1, red);
    const double s2 = block_sum<EXP_THREADS>(d2, red);
    if (tid == 0) {
        a.partials[2 * unit] = s1;
        a.partials[2 * unit + 1] = s2;
    }
}

template <class ST>
hipError_t launch_exp(const stpi_problem *p, const void *s, const void *f, double alpha, void *buf0, void *buf1,
                      DevState *state, double *partials, double x_scale, hipStream_t st) {
    using CT = typename Compute<ST>::type;
    ExpArgs<ST> a;
    a.s = (const ST *)s;
    a.f = (const ST *)f;
    a.buf0 = (ST *)buf0;
    a.buf1 = (ST *)buf1;
    a.state = state;
    a.partials = partials;
    a.x_scale = x_scale;
    a.alpha = (CT)alpha;
    a.T = p->T;
    a.H = p->H;
    a.W = p->W;
    a.rs = p->r_s;
    a.rt = p->r_t;
    double gs[2 * 16 + 1], gt[2 * 8 + 1];
    make_taps(p, gs, gt);
    for (int d = -EXP_RS; d <= EXP_RS; ++d) a.gs[d + EXP_RS] = (CT)gs[d + 16];
    for (int d = -EXP_RT; d <= EXP_RT; ++d) a.gt[d + EXP_RT] = (CT)gt[d + 8];
    const int units = ((p->W + EXP_TILE - 1) / EXP_TILE) * ((p->H + EXP_TILE - 1) / EXP_TILE) * p->T;
    hipLaunchKernelGGL(exp_step_kernel<ST>, dim3(units), dim3(EXP_THREADS), 0, st, a);
    return hipGetLastError();
}

int exp_units(const stpi_problem *p) {
    return ((p->W + EXP_TILE - 1) / EXP_TILE) * ((p->H + EXP_TILE - 1) / EXP_TILE) * p->T;
}

size_t exp_ws_total(const stpi_problem *p, size_t *partials_off, size_t *buf_off) {
    const size_t elem = p->dtype == STPI_F64 ? 8 : 4;
    const size_t cap = std::max((size_t)exp_units(p), (size_t)NORM_BLOCKS_HOST);
    *partials_off = 256;
    *buf_off = 256 + ((cap * 2 * sizeof(double) + 255) & ~(size_t)255);
    return *buf_off + (((size_t)p->T * p->H * p->W * elem + 255) & ~(size_t)255);
}

int exp_check(const stpi_problem *p, double alpha) {
    int rc = validate_problem(p);
    if (rc) return rc;
    if (p->dtype != STPI_F32 && p->dtype != STPI_F64) return fail(STPI_EUNSUPPORTED, "exact affinity: float or double");
    if (p->r_s > EXP_RS || p->r_t > EXP_RT)
        return fail(STPI_EUNSUPPORTED, "exact affinity: radii up to (%d, %d)", EXP_RS, EXP_RT);
    if (!(alpha >= 0.0) || !std::isfinite(alpha)) return fail(STPI_EINVAL, "alpha must be finite and >= 0");
    return STPI_OK;
}

hipError_t exp_launch(const stpi_problem *p, const void *s, const void *f, double alpha, void *b0, void *b1,
                      DevState *state, double *partials, double x_scale, hipStream_t st) {
    return p->dtype == STPI_F64 ? launch_exp<double>(p, s, f, alpha, b0, b1, state, partials, x_scale, st)
                                : launch_exp<float>(p, s, f, alpha, b0, b1, state, partials, x_scale, st);
}

}  // namespace
}  // namespace stpi

using namespace stpi;

extern "C" {

size_t stpi_exp_workspace_bytes(const stpi_problem *p) {
    if (exp_check(p, 0.0) != STPI_OK) return 0;
    size_t a, b;
    return exp_ws_total(p, &a, &b);
}

int stpi_exp_step(const stpi_problem *p, const void *s, const void *f, double alpha, const void *x, double x_scale,
                  void *z, double *d_sums, void *ws, size_t ws_bytes, void *stream) {
    clear_error();
    int rc = exp_check(p, alpha);
    if (rc) return rc;
    if (!s || !f || !x || !z || !d_sums) return fail(STPI_EINVAL, "NULL buffer");
    if (z == s || z == f || z == x) return fail(STPI_EINVAL, "z must not alias s, f or x");
    if (!std::isfinite(x_scale)) return fail(STPI_EINVAL, "x_scale must be finite");
    size_t poff, boff;
    const size_t total = exp_ws_total(p, &poff, &boff);
    if (!ws || ws_bytes < total) return fail(STPI_EWORKSPACE, "exact-affinity workspace needs %zu bytes", total);
    hipStream_t st = (hipStream_t)stream;
    double *partials = (double *)((char *)ws + poff);
    hipError_t e = exp_launch(p, s, f, alpha, const_cast<void *>(x), z, nullptr, partials, x_scale, st);
    if (e == hipSuccess) e = launch_step_sums(partials, exp_units(p), x_scale, d_sums, st);
    return e == hipSuccess ? STPI_OK : hip_fail(e, "exact-affinity step");
}

int stpi_exp_iterate(const stpi_problem *p, const void *s, const void *f, double alpha, void *x, int init,
                     int max_iters, double tol, void *ws, size_t ws_bytes, stpi_result *out, void *stream) {
    clear_error();
    int rc = exp_check(p, alpha);
    if (rc) return rc;
    if (!s || !f || !x || !out) return fail(STPI_EINVAL, "NULL buffer or result");
    if (x == s || x == f) return fail(STPI_EINVAL, "x must not alias s or f");
    if (max_iters < 0) return fail(STPI_EINVAL, "max_iters must be >= 0");
    if (init != 0 && init != 1) return fail(STPI_EINVAL, "init must be 0 (use x) or 1 (uniform)");
    if (!std::isfinite(tol)) return fail(STPI_EINVAL, "tol must be finite");
    size_t poff, boff;
    const size_t total = exp_ws_total(p, &poff, &boff);
    if (!ws || ws_bytes < total) return fail(STPI_EWORKSPACE, "exact-affinity workspace needs %zu bytes", total);
    std::memset(out, 0, sizeof(*out));
    hipStream_t st = (hipStream_t)stream;
    const DtypeOps *ops = ops_for(p->dtype);
    const size_t N = (size_t)p->T * p->H * p->W;
    DevState *state = (DevState *)ws;
    double *partials = (double *)((char *)ws + poff);
    void *buf1 = (char *)ws + boff;
    hipError_t e;
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
    DevState hs;
    for (int done = 0; done < max_iters;) {
        const int n = tol > 0.0 ? std::min(CHAIN_CHUNK, max_iters - done) : max_iters;
        for (int k = 0; k < n; ++k) {
            if ((e = exp_launch(p, s, f, alpha, x, buf1, state, partials, 1.0, st)) != hipSuccess)
                return hip_fail(e, "exact-affinity step");
            if ((e = launch_finalize(partials, exp_units(p), state, st)) != hipSuccess)
                return hip_fail(e, "finalize");
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
    out->status = (hs.flags & FLAG_NONFINITE) ? STPI_ENONFINITE : (hs.flags & FLAG_ZERO) ? STPI_EZERO_NORM : 0;
    if (out->status) return fail(out->status, "iteration stopped after %d steps: %s", hs.iters,
                                 stpi_status_string(out->status));
    return STPI_OK;
}

}  // extern "C"
