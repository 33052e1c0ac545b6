// C ABI of the differentiation path: tape steps, adjoint steps, channel
// combination, normalisation, inner product and the BCE loss.
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstring>

#include "../../include/stpi.h"
#include "host_internal.hpp"

namespace stpi {

constexpr int AUX_BLOCKS_HOST = 512;  // grid of the reduction kernels (matches AUX_BLOCKS)

static int check_aux(int64_t n, int dtype, size_t ws_bytes, const void *ws, bool need_ws) {
    if (n < 1) return fail(STPI_EINVAL, "n must be >= 1");
    if (!ops_for(dtype)) return fail(STPI_EINVAL, "unknown dtype %d", dtype);
    if (need_ws && (!ws || ws_bytes < (size_t)STPI_AUX_WS_BYTES))
        return fail(STPI_EWORKSPACE, "auxiliary workspace needs %d bytes", STPI_AUX_WS_BYTES);
    return STPI_OK;
}

const AdjVariant *choose_adj_variant(const stpi_problem *p) {
    const DtypeOps *ops = ops_for(p->dtype);
    const AdjVariant *best = nullptr;
    int best_cost = 1 << 30;
    for (int i = 0; i < ops->nadj; ++i) {
        const AdjVariant &v = ops->adj_variants[i];
        if (v.RS < p->r_s || v.RT < p->r_t) continue;
        const int c = 2 * (2 * v.RS + 1) + (2 * v.RT + 1);
        if (c < best_cost) {
            best_cost = c;
            best = &v;
        }
    }
    return best;
}

// Frame segments of an adjoint launch (one workgroup per CU): as the forward
// step's, at least 4 r_t frames long while the tiles leave CUs idle, and a
// tile left whole split where that shortens its slowest segment.
int adj_segments(const AdjVariant &v, const stpi_problem *p) {
    const int tiles = ((p->W + v.TW - 1) / v.TW) * ((p->H + v.TH - 1) / v.TH);
    const int rt = v.RT > 0 ? v.RT : 1;
    int nseg = std::min(std::min(device_cus() / tiles, p->T / (4 * rt)), 4);
    if (nseg < 1) nseg = 1;
    if (nseg == 1) nseg = split_short_tiles(tiles, p->T, v.RT);
    return nseg;
}

int adj_grid_blocks(const AdjVariant &v, const stpi_problem *p) {
    return ((p->W + v.TW - 1) / v.TW) * ((p->H + v.TH - 1) / v.TH) * adj_segments(v, p);
}

}  // namespace stpi

using namespace stpi;

extern "C" {

int stpi_train_init(const stpi_problem *p, void *x0, double *norm0, void *stream) {
    clear_error();
    int rc = validate_problem(p);
    if (rc) return rc;
    if (!x0 || !norm0) return fail(STPI_EINVAL, "NULL buffer");
    const size_t N = (size_t)p->T * p->H * p->W;
    hipError_t e = ops_for(p->dtype)->train_init(N, x0, norm0, (hipStream_t)stream);
    return e == hipSuccess ? STPI_OK : hip_fail(e, "train init");
}

int stpi_train_step(const stpi_problem *p, const void *f, const void *z_in, const double *norm_in, void *z_out,
                    void *v_out, double *norm_out, void *ws, size_t ws_bytes, void *stream) {
    clear_error();
    int rc = validate_problem(p);
    if (rc) return rc;
    if (!f || !z_in || !norm_in || !z_out || !norm_out) return fail(STPI_EINVAL, "NULL buffer");
    if (z_out == z_in || z_out == f || (v_out && (v_out == z_in || v_out == f || v_out == z_out)))
        return fail(STPI_EINVAL, "outputs must not alias inputs");
    const WsLayout L = layout_for(p);
    if (!ws || ws_bytes < L.total) return fail(STPI_EWORKSPACE, "workspace needs %zu bytes", L.total);
    const Variant *v = choose_variant(p, forced_variant(), false);
    if (!v) return fail(STPI_EUNSUPPORTED, "no compiled kernel for radii (%d, %d)", p->r_s, p->r_t);
    hipStream_t s = (hipStream_t)stream;
    FwdLaunch FL;
    std::memset(&FL, 0, sizeof(FL));
    FL.f = f;
    FL.buf0 = const_cast<void *>(z_in);
    FL.buf1 = z_out;
    FL.x_scale = 1.0;
    FL.norm_in = norm_in;
    FL.vout = v_out;
    FL.partials = (double *)((char *)ws + L.partials_off);
    FL.T = p->T;
    FL.H = p->H;
    FL.W = p->W;
    FL.nseg = segments_for(*v, p);
    make_taps(p, FL.gs, FL.gt);
    hipError_t e = v->launch(FL, s);
    if (e != hipSuccess) return hip_fail(e, "train step launch");
    e = launch_norm_finalize(FL.partials, grid_blocks(*v, p), norm_out, s);
    return e == hipSuccess ? STPI_OK : hip_fail(e, "norm finalize");
}

int stpi_adjoint_step(const stpi_problem *p, const void *f, const void *z_k, const double *norm_k, const void *z_k1,
                      const double *norm_k1, const void *v_k, const void *g_k1, const double *d_k1, void *g_k,
                      void *g_f, double *d_k, void *ws, size_t ws_bytes, void *stream) {
    clear_error();
    int rc = validate_problem(p);
    if (rc) return rc;
    if (!f || !z_k || !norm_k || !z_k1 || !norm_k1 || !v_k || !g_k1 || !d_k1 || !g_k || !g_f || !d_k)
        return fail(STPI_EINVAL, "NULL buffer");
    if (g_k == g_k1 || g_k == g_f || g_k == f || g_k == z_k || g_k == z_k1 || g_k == v_k)
        return fail(STPI_EINVAL, "g_k must not alias another argument");
    const WsLayout L = layout_for(p);
    if (!ws || ws_bytes < L.total) return fail(STPI_EWORKSPACE, "workspace needs %zu bytes", L.total);
    const AdjVariant *v = choose_adj_variant(p);
    if (!v) return fail(STPI_EUNSUPPORTED, "no adjoint kernel for dtype %d, radii (%d, %d)", p->dtype, p->r_s, p->r_t);
    hipStream_t s = (hipStream_t)stream;
    AdjLaunch AL;
    std::memset(&AL, 0, sizeof(AL));
    AL.f = f;
    AL.zk = z_k;
    AL.zk1 = z_k1;
    AL.vk = v_k;
    AL.g1 = g_k1;
    AL.gk = g_k;
    AL.gf = g_f;
    AL.norm_k = norm_k;
    AL.norm_k1 = norm_k1;
    AL.d_k1 = d_k1;
    AL.partials = (double *)((char *)ws + L.partials_off);
    AL.T = p->T;
    AL.H = p->H;
    AL.W = p->W;
    AL.nseg = adj_segments(*v, p);
    make_taps(p, AL.gs, AL.gt);
    hipError_t e = v->launch(AL, s);
    if (e != hipSuccess) return hip_fail(e, "adjoint launch");
    e = launch_sum0_finalize(AL.partials, adj_grid_blocks(*v, p), d_k, s);
    return e == hipSuccess ? STPI_OK : hip_fail(e, "adjoint finalize");
}

int stpi_normalize(int64_t n, int dtype, const void *z, const double *norm, void *x, void *stream) {
    clear_error();
    int rc = check_aux(n, dtype, 0, nullptr, false);
    if (rc) return rc;
    if (!z || !norm || !x) return fail(STPI_EINVAL, "NULL buffer");
    hipError_t e = ops_for(dtype)->scale_by_norm((size_t)n, z, norm, x, (hipStream_t)stream);
    return e == hipSuccess ? STPI_OK : hip_fail(e, "normalize");
}

int stpi_dot(int64_t n, int dtype, const void *a, const double *a_norm, const void *b, double *out, void *ws,
             size_t ws_bytes, void *stream) {
    clear_error();
    int rc = check_aux(n, dtype, ws_bytes, ws, true);
    if (rc) return rc;
    if (!a || !b || !out) return fail(STPI_EINVAL, "NULL buffer");
    hipStream_t s = (hipStream_t)stream;
    double *partials = (double *)ws;
    hipError_t e = ops_for(dtype)->dot((size_t)n, a, b, partials, s);
    if (e == hipSuccess) e = launch_dot_finalize(partials, AUX_BLOCKS_HOST, a_norm, out, s);
    return e == hipSuccess ? STPI_OK : hip_fail(e, "dot");
}

int stpi_combine_fwd(int C, int64_t n, int dtype, const void *fc, const double *w, void *f, void *stream) {
    clear_error();
    int rc = check_aux(n, dtype, 0, nullptr, false);
    if (rc) return rc;
    if (C < 1 || C > STPI_MAX_CHANNELS) return fail(STPI_EINVAL, "C must be in [1, %d]", STPI_MAX_CHANNELS);
    if (!fc || !w || !f) return fail(STPI_EINVAL, "NULL buffer");
    hipError_t e = ops_for(dtype)->combine_fwd(C, (size_t)n, fc, w, f, (hipStream_t)stream);
    return e == hipSuccess ? STPI_OK : hip_fail(e, "combine forward");
}

int stpi_combine_bwd(int C, int64_t n, int dtype, const void *fc, const double *w, const void *g_f, double *g_w,
                     void *ws, size_t ws_bytes, void *stream) {
    clear_error();
    int rc = check_aux(n, dtype, ws_bytes, ws, true);
    if (rc) return rc;
    if (C < 1 || C > STPI_MAX_CHANNELS) return fail(STPI_EINVAL, "C must be in [1, %d]", STPI_MAX_CHANNELS);
    if (!fc || !w || !g_f || !g_w) return fail(STPI_EINVAL, "NULL buffer");
    hipStream_t s = (hipStream_t)stream;
    double *partials = (double *)ws;
    hipError_t e = ops_for(dtype)->combine_bwd(C, (size_t)n, fc, g_f, partials, s);
    if (e == hipSuccess) e = launch_combine_bwd_finalize(C, AUX_BLOCKS_HOST, partials, w, g_w, s);
    return e == hipSuccess ? STPI_OK : hip_fail(e, "combine backward");
}

int stpi_bce(int64_t n, int dtype, const void *x, const uint8_t *gt, double *loss, void *g_x, void *ws,
             size_t ws_bytes, void *stream) {
    clear_error();
    int rc = check_aux(n, dtype, ws_bytes, ws, true);
    if (rc) return rc;
    if (!x || !gt || !loss || !g_x) return fail(STPI_EINVAL, "NULL buffer");
    if (g_x == x) return fail(STPI_EINVAL, "g_x must not alias x");
    hipStream_t s = (hipStream_t)stream;
    const DtypeOps *ops = ops_for(dtype);
    double *partials = (double *)ws;
    double *scalars = partials + 2 * AUX_BLOCKS_HOST;
    hipError_t e = ops->maxarg((size_t)n, x, partials, s);
    if (e == hipSuccess) e = launch_max_finalize(AUX_BLOCKS_HOST, partials, scalars, s);
    if (e == hipSuccess) e = ops->bce((size_t)n, x, gt, scalars, g_x, partials, s);
    if (e == hipSuccess) e = ops->bce_finalize((size_t)n, AUX_BLOCKS_HOST, partials, scalars, g_x, loss, s);
    return e == hipSuccess ? STPI_OK : hip_fail(e, "bce");
}

int stpi_adamw(int64_t n, int dtype, void *w, const void *g, void *m, void *v, void *vmax, int step, double lr,
               double beta1, double beta2, double eps, double weight_decay, int amsgrad, void *stream) {
    clear_error();
    if (n < 1) return fail(STPI_EINVAL, "n must be >= 1");
    if (dtype != STPI_F32 && dtype != STPI_F64) return fail(STPI_EINVAL, "AdamW works on float or double parameters");
    if (!w || !g || !m || !v || (amsgrad && !vmax)) return fail(STPI_EINVAL, "NULL buffer");
    if (step < 1) return fail(STPI_EINVAL, "step is 1-based");
    if (!(lr >= 0.0) || !(beta1 >= 0.0 && beta1 < 1.0) || !(beta2 >= 0.0 && beta2 < 1.0) || !(eps > 0.0))
        return fail(STPI_EINVAL, "bad AdamW hyper-parameters");
    const double bc1 = 1.0 - std::pow(beta1, step), bc2 = 1.0 - std::pow(beta2, step);
    hipError_t e = launch_adamw(dtype, n, w, g, m, v, vmax, lr, beta1, beta2, eps, weight_decay, bc1, bc2,
                                amsgrad ? 1 : 0, (hipStream_t)stream);
    return e == hipSuccess ? STPI_OK : hip_fail(e, "adamw");
}

}  // extern "C"
