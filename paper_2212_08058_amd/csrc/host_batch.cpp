// C ABI of the batched path: plans, the batched iteration chain and its graph.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstring>
#include <numeric>
#include <vector>

#include "../../include/stpi.h"
#include "host_internal.hpp"

struct stpi_plan {
    stpi_problem proto;  // sigmas, radii, dtype (T, H, W unused)
    int nclips = 0, ntiles = 0, grid = 0;
    const stpi::BatchVariant *v = nullptr;
    stpi::ClipDesc *d_clips = nullptr;
    stpi::TileDesc *d_tiles = nullptr;
    int32_t *d_order = nullptr;  // clip indices in tile-list order
    std::vector<stpi::ClipDesc> clips;  // host copy, in the caller's order
    int64_t extent = 0;                 // elements the flat buffers must hold
    size_t ws_state_off = 0, ws_active_off = 0, ws_partials_off = 0, ws_buf_off = 0, ws_total = 0;
    // captured chains: (f, x, ws, init, max_iters, tol, stream) -> graph
    struct G {
        const void *f;
        void *x, *ws;
        int init, max_iters;
        double tol;
        hipStream_t s;
        int part;
        hipGraphExec_t exec;
        hipEvent_t launched;  // recorded after every launch: eviction waits for it
    };
    stpi::BatchCtl *poll = nullptr;  // pinned copy of the chain counters (stop-flag poll)
    hipEvent_t poll_ev = nullptr;
    std::vector<G> graphs;
};

namespace stpi {

static const BatchVariant *choose_batch_variant(const stpi_problem *proto, const std::vector<ClipDesc> &clips) {
    const DtypeOps *ops = ops_for(proto->dtype);
    // Prefer the variant the autotuner picked for the frame size carrying the
    // most voxels; otherwise the cheapest eligible one by the tap-count model.
    std::vector<std::pair<int64_t, std::pair<int, int>>> by_shape;
    for (const auto &c : clips) {
        bool found = false;
        for (auto &e : by_shape)
            if (e.second.first == c.H && e.second.second == c.W) {
                e.first += (int64_t)c.T * c.H * c.W;
                found = true;
            }
        if (!found) by_shape.push_back({(int64_t)c.T * c.H * c.W, {c.H, c.W}});
    }
    std::sort(by_shape.begin(), by_shape.end(), [](auto &a, auto &b) { return a.first > b.first; });
    if (!by_shape.empty()) {
        stpi_problem q = *proto;
        q.T = 64;
        q.H = by_shape[0].second.first;
        q.W = by_shape[0].second.second;
        const int tv = tuned_variant(&q);
        if (tv >= 0 && tv < ops->nvariants) {
            const Variant &fv = ops->variants[tv];
            for (int i = 0; i < ops->nbatch; ++i) {
                const BatchVariant &b = ops->batch_variants[i];
                if (b.RS == fv.RS && b.RT == fv.RT && b.TH == fv.TH && b.TW == fv.TW && b.NTHR == fv.NTHR &&
                    b.RY == fv.RY && b.QX == fv.QX && b.PIPE == (fv.PIPE == 3 ? 3 : (fv.PIPE ? 1 : 0)))
                    return &b;
            }
        }
    }
    const BatchVariant *best = nullptr;
    double best_cost = 1e300;
    for (int i = 0; i < ops->nbatch; ++i) {
        const BatchVariant &b = ops->batch_variants[i];
        if (b.RS < proto->r_s || b.RT < proto->r_t) continue;
        double cost = 0.0;
        // the single-clip model (matrix-core variants: product form, see variant_cost)
        const double taps = b.PIPE == 3 ? ((b.RS > 8 ? 42.0 : 30.0) + 2.0 * (2.0 * b.RT + 1)) *
                                              (b.blocks_per_cu() >= 2 ? 0.9 : 1.0)
                                        : (2.0 * b.RS + 1) * (1.0 + 2.0 * b.RS / b.TW) + (2.0 * b.RS + 1) +
                                              (2.0 * b.RT + 1);
        for (const auto &c : clips) {
            const double gx = std::ceil((double)c.W / b.TW), gy = std::ceil((double)c.H / b.TH);
            cost += gx * gy * b.TW * b.TH * (double)c.T * taps;
        }
        if (cost < best_cost) {
            best_cost = cost;
            best = &b;
        }
    }
    return best;
}

// part: 0 everything, 1 init + CHAIN_CHUNK steps, 2 CHAIN_CHUNK steps, 3 final normalisation
static int enqueue_batch(stpi_plan *P, const void *f, void *x, void *ws, int init, int max_iters, double tol,
                         hipStream_t s, int part = 0) {
    const DtypeOps *ops = ops_for(P->proto.dtype);
    char *w = (char *)ws;
    BatchCtl *ctl = (BatchCtl *)w;
    DevState *states = (DevState *)(w + P->ws_state_off);
    double *partials = (double *)(w + P->ws_partials_off);
    int32_t *active_clip = (int32_t *)(w + P->ws_active_off);
    int32_t *active_cum = active_clip + P->nclips;
    void *buf1 = w + P->ws_buf_off;
    hipError_t e;
    auto compact = [&]() -> hipError_t {
        return launch_batch_compact(states, P->d_clips, P->d_order, P->nclips, active_clip, active_cum, ctl, s);
    };
    // matrix-core variants run every step in product form (a chain of no steps never launches one)
    const int pform = P->v->PIPE == 3 && max_iters > 0 ? 1 : 0;
    auto tail = [&]() -> hipError_t {
        return pform ? ops->batch_from_product(x, buf1, f, P->d_clips, states, P->nclips, s)
                     : ops->batch_normalize(x, buf1, P->d_clips, states, P->nclips, s);
    };
    if (part == 3) {
        if ((e = tail()) != hipSuccess) return hip_fail(e, "batch normalize");
        return STPI_OK;
    }
    if (part <= 1) {
        if ((e = launch_batch_init(states, P->d_clips, P->nclips, tol, max_iters, init == 1 ? 1 : 0,
                                   init == 2 ? 1 : 0, pform, ctl, s)) != hipSuccess)
            return hip_fail(e, "batch init");
        if (init == 1) {
            // product form: the first step stages f itself
            if (!pform && (e = ops->batch_fill(x, P->d_clips, P->nclips, s)) != hipSuccess)
                return hip_fail(e, "batch fill");
        } else {
            if ((e = ops->batch_sumsq(x, P->d_clips, P->nclips, partials, s)) != hipSuccess)
                return hip_fail(e, "batch norm");
            if ((e = launch_batch_state_from_norm(partials, states, P->nclips, ctl, s)) != hipSuccess)
                return hip_fail(e, "batch norm finalize");
        }
        if (P->v->PIPE == 3 && (e = ops->batch_bound(f, P->d_clips, states, P->nclips, s)) != hipSuccess)
            return hip_fail(e, "batch operand bound");
        if (pform && init != 1 &&
            (e = ops->batch_to_product(f, x, buf1, P->d_clips, states, P->nclips, s)) != hipSuccess)
            return hip_fail(e, "batch product-form start");
        if ((e = compact()) != hipSuccess) return hip_fail(e, "batch active list");
    }
    BatchLaunch BL;
    std::memset(&BL, 0, sizeof(BL));
    BL.f = f;
    BL.buf0 = x;
    BL.buf1 = buf1;
    BL.states = states;
    BL.clips = P->d_clips;
    BL.tiles = P->d_tiles;
    BL.ctl = ctl;
    BL.partials = partials;
    BL.active_clip = active_clip;
    BL.active_cum = active_cum;
    BL.ntiles = P->ntiles;
    BL.nclips = P->nclips;
    BL.grid = P->grid;
    make_taps(&P->proto, BL.gs, BL.gt);
    const int steps = part == 0 ? max_iters : CHAIN_CHUNK;
    for (int k = 0; k < steps; ++k) {
        if ((e = P->v->launch(BL, s)) != hipSuccess) return hip_fail(e, "batch step");
        if ((e = launch_batch_finalize(partials, P->d_clips, states, P->nclips, ctl, s)) != hipSuccess)
            return hip_fail(e, "batch finalize");
        // the rise check fires after the second step; plain-form clips that
        // restart need their buffer refilled (product-form ones stage f)
        if (init == 2 && !pform && part <= 1 && k == 1 &&
            (e = ops->batch_refill(x, buf1, P->d_clips, states, P->nclips, s)) != hipSuccess)
            return hip_fail(e, "batch refill");
        if ((e = compact()) != hipSuccess) return hip_fail(e, "batch active list");
    }
    if (part == 0 && (e = tail()) != hipSuccess) return hip_fail(e, "batch normalize");
    return STPI_OK;
}

}  // namespace stpi

using namespace stpi;

extern "C" {

int stpi_batch_plan(const stpi_clip *clips, int nclips, float sigma_s, float sigma_t, int r_s, int r_t, int dtype,
                    stpi_plan **out) {
    clear_error();
    if (!clips || nclips < 1 || !out) return fail(STPI_EINVAL, "need at least one clip and an output pointer");
    *out = nullptr;
    stpi_problem proto;
    proto.T = proto.H = proto.W = 1;
    proto.sigma_s = sigma_s;
    proto.sigma_t = sigma_t;
    proto.r_s = r_s;
    proto.r_t = r_t;
    proto.dtype = dtype;
    int rc = validate_problem(&proto);
    if (rc) return rc;
    std::vector<ClipDesc> cds(nclips);
    int64_t extent = 0;
    for (int i = 0; i < nclips; ++i) {
        stpi_problem q = proto;
        q.T = clips[i].T;
        q.H = clips[i].H;
        q.W = clips[i].W;
        if ((rc = validate_problem(&q))) return fail(rc, "clip %d: %s", i, stpi_last_error());
        if (clips[i].offset < 0) return fail(STPI_EINVAL, "clip %d: negative offset", i);
        cds[i].offset = clips[i].offset;
        cds[i].T = clips[i].T;
        cds[i].H = clips[i].H;
        cds[i].W = clips[i].W;
        extent = std::max(extent, clips[i].offset + (int64_t)clips[i].T * clips[i].H * clips[i].W);
    }
    // clips must not overlap
    std::vector<int> order(nclips);
    std::iota(order.begin(), order.end(), 0);
    std::sort(order.begin(), order.end(), [&](int a, int b) { return cds[a].offset < cds[b].offset; });
    for (int i = 1; i < nclips; ++i) {
        const ClipDesc &p = cds[order[i - 1]];
        if (p.offset + (int64_t)p.T * p.H * p.W > cds[order[i]].offset)
            return fail(STPI_EINVAL, "clips %d and %d overlap", order[i - 1], order[i]);
    }
    const BatchVariant *v = choose_batch_variant(&proto, cds);
    if (!v) return fail(STPI_EUNSUPPORTED, "no batched kernel for dtype %d, radii (%d, %d)", dtype, r_s, r_t);
    // tile list: longest clips first, each clip's tiles contiguous, row-major
    std::vector<int> by_len(nclips);
    std::iota(by_len.begin(), by_len.end(), 0);
    std::stable_sort(by_len.begin(), by_len.end(), [&](int a, int b) {
        const int64_t wa = (int64_t)cds[a].T * ((cds[a].H + v->TH - 1) / v->TH) * ((cds[a].W + v->TW - 1) / v->TW);
        const int64_t wb = (int64_t)cds[b].T * ((cds[b].H + v->TH - 1) / v->TH) * ((cds[b].W + v->TW - 1) / v->TW);
        return cds[a].T > cds[b].T || (cds[a].T == cds[b].T && wa > wb);
    });
    std::vector<TileDesc> tiles;
    for (int c : by_len) {
        cds[c].tile_begin = (int)tiles.size();
        const int nbx = (cds[c].W + v->TW - 1) / v->TW, nby = (cds[c].H + v->TH - 1) / v->TH;
        for (int ty = 0; ty < nby; ++ty)
            for (int tx = 0; tx < nbx; ++tx) tiles.push_back(TileDesc{c, tx * v->TW, ty * v->TH, 0});
        cds[c].tile_end = (int)tiles.size();
    }
    stpi_plan *P = new stpi_plan();
    P->proto = proto;
    P->nclips = nclips;
    P->ntiles = (int)tiles.size();
    P->v = v;
    P->clips = cds;
    P->extent = extent;
    int dev = 0, cus = 256;
    hipDeviceProp_t prop;
    if (hipGetDevice(&dev) == hipSuccess && hipGetDeviceProperties(&prop, dev) == hipSuccess)
        cus = prop.multiProcessorCount;
    P->grid = cus * v->blocks_per_cu();
    hipError_t e = hipMalloc((void **)&P->d_clips, sizeof(ClipDesc) * nclips);
    if (e == hipSuccess) e = hipMalloc((void **)&P->d_tiles, sizeof(TileDesc) * tiles.size());
    if (e == hipSuccess) e = hipMalloc((void **)&P->d_order, sizeof(int32_t) * nclips);
    if (e == hipSuccess) e = hipMemcpy(P->d_order, by_len.data(), sizeof(int32_t) * nclips, hipMemcpyHostToDevice);
    if (e == hipSuccess)
        e = hipMemcpy(P->d_clips, cds.data(), sizeof(ClipDesc) * nclips, hipMemcpyHostToDevice);
    if (e == hipSuccess)
        e = hipMemcpy(P->d_tiles, tiles.data(), sizeof(TileDesc) * tiles.size(), hipMemcpyHostToDevice);
    if (e != hipSuccess) {
        stpi_plan_destroy(P);
        return hip_fail(e, "plan tables");
    }
    const size_t elem = ops_for(dtype)->elem;
    P->ws_state_off = 256;
    size_t off = P->ws_state_off + ((sizeof(DevState) * nclips + 255) & ~(size_t)255);
    P->ws_active_off = off;
    off += ((sizeof(int32_t) * 2 * nclips + 255) & ~(size_t)255);
    P->ws_partials_off = off;
    const size_t npart = std::max((size_t)P->ntiles, (size_t)nclips * BATCH_NORM_BLOCKS);
    off += ((npart * 2 * sizeof(double) + 255) & ~(size_t)255);
    P->ws_buf_off = off;
    P->ws_total = off + (((size_t)extent * elem + 255) & ~(size_t)255);
    *out = P;
    return STPI_OK;
}

size_t stpi_batch_workspace_bytes(const stpi_plan *plan) { return plan ? plan->ws_total : 0; }

int stpi_batch_info(const stpi_plan *plan, int32_t info[11]) {
    clear_error();
    if (!plan || !info) return fail(STPI_EINVAL, "NULL plan or info");
    const BatchVariant *v = plan->v;
    info[0] = plan->nclips;
    info[1] = plan->ntiles;
    info[2] = plan->grid;
    info[3] = v->RS;
    info[4] = v->RT;
    info[5] = v->TH;
    info[6] = v->TW;
    info[7] = v->NTHR;
    info[8] = v->RY;
    info[9] = v->QX;
    info[10] = v->PIPE;
    return STPI_OK;
}

int stpi_batch_iterate(stpi_plan *plan, const void *f, void *x, int init, int max_iters, double tol, void *ws,
                       size_t ws_bytes, stpi_result *per_clip, void *stream) {
    clear_error();
    if (!plan || !f || !x || !per_clip) return fail(STPI_EINVAL, "NULL plan, buffer or result");
    if (f == x) return fail(STPI_EINVAL, "x must not alias f");
    if (max_iters < 0) return fail(STPI_EINVAL, "max_iters must be >= 0");
    if (init < 0 || init > 2)
        return fail(STPI_EINVAL, "init must be 0 (use x), 1 (uniform) or 2 (use x, rise check per clip)");
    if (!std::isfinite(tol)) return fail(STPI_EINVAL, "tol must be finite");
    if (!ws || ws_bytes < plan->ws_total)
        return fail(STPI_EWORKSPACE, "batch workspace needs %zu bytes", plan->ws_total);
    hipStream_t s = (hipStream_t)stream;
    int rc;
    auto run = [&](int part) -> int {
        if (s == nullptr) return enqueue_batch(plan, f, x, ws, init, max_iters, tol, s, part);
        hipGraphExec_t exec = nullptr;
        hipEvent_t launched = nullptr;
        for (auto &g : plan->graphs)
            if (g.f == f && g.x == x && g.ws == ws && g.init == init && g.max_iters == max_iters && g.tol == tol &&
                g.s == s && g.part == part) {
                exec = g.exec;
                launched = g.launched;
            }
        hipError_t e;
        if (!exec) {
            if ((e = hipStreamBeginCapture(s, hipStreamCaptureModeThreadLocal)) != hipSuccess)
                return hip_fail(e, "begin capture");
            const int rc2 = enqueue_batch(plan, f, x, ws, init, max_iters, tol, s, part);
            hipGraph_t graph = nullptr;
            e = hipStreamEndCapture(s, &graph);
            if (rc2) {
                if (graph) (void)hipGraphDestroy(graph);
                return rc2;
            }
            if (e != hipSuccess) return hip_fail(e, "end capture");
            e = hipGraphInstantiate(&exec, graph, nullptr, nullptr, 0);
            (void)hipGraphDestroy(graph);
            if (e != hipSuccess) return hip_fail(e, "graph instantiate");
            if ((e = hipEventCreateWithFlags(&launched, hipEventDisableTiming)) != hipSuccess) {
                (void)hipGraphExecDestroy(exec);
                return hip_fail(e, "graph event");
            }
            if (plan->graphs.size() >= 16) {
                // the oldest graph may still be queued: wait for its last launch
                (void)hipEventSynchronize(plan->graphs.front().launched);
                (void)hipGraphExecDestroy(plan->graphs.front().exec);
                (void)hipEventDestroy(plan->graphs.front().launched);
                plan->graphs.erase(plan->graphs.begin());
            }
            plan->graphs.push_back({f, x, ws, init, max_iters, tol, s, part, exec, launched});
        }
        if ((e = hipGraphLaunch(exec, s)) != hipSuccess) return hip_fail(e, "graph launch");
        if ((e = hipEventRecord(launched, s)) != hipSuccess) return hip_fail(e, "graph event");
        return STPI_OK;
    };
    // Long tolerance runs replay CHAIN_CHUNK steps at a time and stop once
    // every clip is done (checked one chunk behind, as stpi_iterate does).
    if (!(tol > 0.0 && max_iters > 2 * CHAIN_CHUNK)) {
        if ((rc = run(0))) return rc;
    } else {
        hipError_t e;
        if (!plan->poll && hipHostMalloc((void **)&plan->poll, sizeof(BatchCtl), hipHostMallocDefault) != hipSuccess) {
            plan->poll = nullptr;
            return fail(STPI_EHIP, "pinned poll buffer");
        }
        if (!plan->poll_ev && (e = hipEventCreateWithFlags(&plan->poll_ev, hipEventDisableTiming)) != hipSuccess)
            return hip_fail(e, "poll event");
        if ((rc = run(1))) return rc;
        for (int issued = CHAIN_CHUNK; issued < max_iters; issued += CHAIN_CHUNK) {
            if ((e = hipMemcpyAsync(plan->poll, ws, sizeof(BatchCtl), hipMemcpyDeviceToHost, s)) != hipSuccess)
                return hip_fail(e, "counter poll");
            if ((e = hipEventRecord(plan->poll_ev, s)) != hipSuccess) return hip_fail(e, "poll event");
            if ((rc = run(2))) return rc;
            if ((e = hipEventSynchronize(plan->poll_ev)) != hipSuccess) return hip_fail(e, "poll wait");
            if (plan->poll->done_clips >= (uint32_t)plan->nclips) break;
        }
        if ((rc = run(3))) return rc;
    }
    std::vector<DevState> hs(plan->nclips);
    hipError_t e = hipMemcpyAsync(hs.data(), (char *)ws + plan->ws_state_off, sizeof(DevState) * plan->nclips,
                                  hipMemcpyDeviceToHost, s);
    if (e == hipSuccess) e = hipStreamSynchronize(s);
    if (e != hipSuccess) return hip_fail(e, "batch readback");
    int worst = STPI_OK;
    for (int i = 0; i < plan->nclips; ++i) {
        stpi_result &r = per_clip[i];
        r.iters = hs[i].iters;
        r.converged = hs[i].converged;
        r.flags = hs[i].flags;
        r.residual = hs[i].residual;
        r.lambda = hs[i].lambda;
        r.rayleigh = hs[i].rayleigh;
        r.first_residuals[0] = hs[i].first_res[0];
        r.first_residuals[1] = hs[i].first_res[1];
        r.status = (hs[i].flags & FLAG_NONFINITE) ? STPI_ENONFINITE : (hs[i].flags & FLAG_ZERO) ? STPI_EZERO_NORM : 0;
        if (r.status && !worst) worst = r.status;
    }
    if (worst) return fail(worst, "at least one clip stopped with: %s", stpi_status_string(worst));
    return STPI_OK;
}

void stpi_plan_destroy(stpi_plan *plan) {
    if (!plan) return;
    for (auto &g : plan->graphs) {
        (void)hipEventSynchronize(g.launched);
        (void)hipGraphExecDestroy(g.exec);
        (void)hipEventDestroy(g.launched);
    }
    if (plan->poll) (void)hipHostFree(plan->poll);
    if (plan->poll_ev) (void)hipEventDestroy(plan->poll_ev);
    if (plan->d_clips) (void)hipFree(plan->d_clips);
    if (plan->d_tiles) (void)hipFree(plan->d_tiles);
    if (plan->d_order) (void)hipFree(plan->d_order);
    delete plan;
}

}  // extern "C"
