// Host side of libstpi: argument validation, filter taps, kernel selection,
// workspace layout and the C ABI declared in include/stpi.h.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <mutex>
#include <string>
#include <vector>

#include "../../include/stpi.h"
#include "dtype_ops.hpp"
#include "host_internal.hpp"

namespace stpi {

static thread_local std::string g_last_error;

int fail(int status, const char *fmt, ...) {
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof(buf), fmt, ap);
    va_end(ap);
    g_last_error = buf;
    return status;
}

int hip_fail(hipError_t e, const char *where) {
    return fail(STPI_EHIP, "%s: %s", where, hipGetErrorString(e));
}

void clear_error() { g_last_error.clear(); }

const DtypeOps *ops_for(int dtype) {
    switch (dtype) {
        case STPI_F32: return dtype_ops_f32();
        case STPI_BF16: return dtype_ops_bf16();
        case STPI_F64: return dtype_ops_f64();
        default: return nullptr;
    }
}

int validate_problem(const stpi_problem *p) {
    if (!p) return fail(STPI_EINVAL, "problem is NULL");
    if (p->T < 1 || p->H < 1 || p->W < 1)
        return fail(STPI_EINVAL, "volume must be at least 1x1x1 (got %dx%dx%d)", p->T, p->H, p->W);
    if (!(p->sigma_s > 0.0f) || !(p->sigma_t > 0.0f) || !std::isfinite(p->sigma_s) || !std::isfinite(p->sigma_t))
        return fail(STPI_EINVAL, "sigmas must be finite and > 0");
    if (p->r_s < 0 || p->r_t < 0) return fail(STPI_EINVAL, "radii must be >= 0");
    if (p->r_s > STPI_MAX_RS || p->r_t > STPI_MAX_RT)
        return fail(STPI_EUNSUPPORTED, "radii (%d, %d) exceed the compiled maximum (%d, %d)", p->r_s, p->r_t,
                    STPI_MAX_RS, STPI_MAX_RT);
    if (!ops_for(p->dtype)) return fail(STPI_EINVAL, "unknown dtype %d", p->dtype);
    if ((int64_t)p->H * p->W > (int64_t)1 << 30)
        return fail(STPI_EUNSUPPORTED, "frame of %d x %d voxels is too large", p->H, p->W);
    return STPI_OK;
}

// Taps exp(-d^2 / (2 sigma^2)) for |d| <= r, centred at index 16 (space) / 8
// (time), zero beyond the radius. The centre tap is 1 (unnormalised kernel).
void make_taps(const stpi_problem *p, double *gs, double *gt) {
    for (int i = 0; i < 2 * 16 + 1; ++i) gs[i] = 0.0;
    for (int i = 0; i < 2 * 8 + 1; ++i) gt[i] = 0.0;
    const double ss = (double)p->sigma_s, stt = (double)p->sigma_t;
    for (int d = -p->r_s; d <= p->r_s; ++d) gs[d + 16] = std::exp(-(double)(d * d) / (2.0 * ss * ss));
    for (int d = -p->r_t; d <= p->r_t; ++d) gt[d + 8] = std::exp(-(double)(d * d) / (2.0 * stt * stt));
}

static double variant_cost(const Variant &v, const stpi_problem *p) {
    // Taps per voxel plus the y-pass over the x-halo, on the padded tile grid.
    const double gx = std::ceil((double)p->W / v.TW), gy = std::ceil((double)p->H / v.TH);
    const double cover = gx * v.TW * gy * v.TH / ((double)p->W * p->H);
    if (v.PIPE == 3) {
        // matrix-core spatial passes (chains in product form): bound by memory
        // traffic and latency, not by the space radius; in the units of the
        // tap count below, measured at 480 x 854 frames as 42 (margin 16) or
        // 30 (margin 8) plus two per temporal tap, 10% less where two
        // workgroups share a CU
        const double base = v.RS > 8 ? 42.0 : 30.0;
        const double occ = v.blocks_per_cu() >= 2 ? 0.9 : 1.0;
        return (base + 2.0 * (2.0 * v.RT + 1)) * cover * occ;
    }
    const double taps = (2.0 * v.RS + 1) * (1.0 + 2.0 * v.RS / v.TW) + (2.0 * v.RS + 1) + (2.0 * v.RT + 1);
    return taps * cover;
}

const Variant *choose_variant(const stpi_problem *p, int forced_index, bool allow_mfma) {
    const DtypeOps *ops = ops_for(p->dtype);
    if (forced_index >= 0 && forced_index < ops->nvariants && !allow_mfma && ops->variants[forced_index].PIPE == 3)
        forced_index = -1;
    if (forced_index >= 0) {
        if (forced_index >= ops->nvariants) return nullptr;
        const Variant &v = ops->variants[forced_index];
        if (v.RS < p->r_s || v.RT < p->r_t) return nullptr;
        return &v;
    }
    int tuned = tuned_variant(p);
    if (tuned >= 0 && tuned < ops->nvariants) {
        const Variant &v = ops->variants[tuned];
        if (v.RS >= p->r_s && v.RT >= p->r_t && (allow_mfma || v.PIPE != 3)) return &v;
    }
    const Variant *best = nullptr;
    double best_cost = 1e300;
    for (int i = 0; i < ops->nvariants; ++i) {
        const Variant &v = ops->variants[i];
        if (v.RS < p->r_s || v.RT < p->r_t) continue;
        if (v.PIPE == 3 && !allow_mfma) continue;
        const double c = variant_cost(v, p);
        if (c < best_cost) {
            best_cost = c;
            best = &v;
        }
    }
    return best;
}

static int tiles_for(const Variant &v, const stpi_problem *p) {
    return ((p->W + v.TW - 1) / v.TW) * ((p->H + v.TH - 1) / v.TH);
}

int device_cus() {
    static int cus[64] = {0};
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= 64) return 256;
    if (cus[dev] == 0) {
        hipDeviceProp_t prop;
        cus[dev] = hipGetDeviceProperties(&prop, dev) == hipSuccess && prop.multiProcessorCount > 0
                       ? prop.multiProcessorCount
                       : 256;
    }
    return cus[dev];
}

// Phases of the slowest of k frame segments of a T-frame tile: the frame walk
// of the tile loops (FrameWalk: RT input frames staged beyond each inner
// boundary, the last segment walked backward when it starts after frame 0)
// plus the 2 phases that fill the pipeline.
int segment_phases(int T, int RT, int k) {
    int worst = 0;
    for (int s = 0; s < k; ++s) {
        const int t0 = (int)((long)s * T / k), t1 = (int)((long)(s + 1) * T / k);
        const int ts = std::max(t0 - RT, 0), te = std::min(t1 + RT, T);
        const bool rev = t1 == T && t0 > 0;
        worst = std::max(worst, (rev ? te - t0 : t1 - ts) + RT + 2);
    }
    return worst;
}

// A tile that the rules below leave whole: when every segment can have a CU
// of its own, the step takes as long as its slowest segment, so split the
// frames where that lowers the phase count (a whole tile ends with RT
// epilogue-only phases that a split with a backward last segment avoids;
// short clips, e.g. the windows of an online run, gain most).
int split_short_tiles(int tiles, int T, int RT) {
    const int cus = device_cus();
    if (2L * tiles > cus) return 1;
    const int kmax = std::min(std::min(cus / tiles, STPI_NSEG_MAX), T);
    // more segments only for at least two phases fewer (each adds a
    // workgroup that re-stages RT frames)
    int best = 1;
    for (int k = 2; k <= kmax; ++k)
        if (segment_phases(T, RT, k) + 1 < segment_phases(T, RT, best)) best = k;
    return best;
}

// Frame segments per tile. When a clip has fewer tiles than the chip holds
// resident workgroups, each tile's frames are split so that more workgroups
// (with independent barriers) share every CU. A segment re-reads and
// re-filters RT input frames on each inner side, so segments are normally at
// least 4 RT frames long and at most 4 per tile. A launch that would still
// fill less than half of the resident slots (a small clip, e.g. a coarse
// level of a two-level start) is bound by the frame-after-frame latency of
// its few workgroups, not by work: there segments may be as short as 2 RT
// frames and up to STPI_NSEG_MAX per tile.
int segments_for(const Variant &v, const stpi_problem *p) {
    const int tiles = tiles_for(v, p);
    const int resident = device_cus() * v.blocks_per_cu();
    const int rt = v.RT > 0 ? v.RT : 1;
    const int fit = resident / tiles;
    int nseg = std::min(std::min(fit, p->T / (4 * rt)), 4);
    if (nseg < 1) nseg = 1;
    if ((long)tiles * nseg * 2 <= resident) {
        const int small = std::min(std::min(fit, p->T / (2 * rt)), STPI_NSEG_MAX);
        if (small > nseg) nseg = small;
    }
    if (nseg == 1) nseg = split_short_tiles(tiles, p->T, v.RT);
    return nseg;
}

int grid_blocks(const Variant &v, const stpi_problem *p) { return tiles_for(v, p) * segments_for(v, p); }

// Workspace: [state 256 B][partials][ping-pong volume]. The partials area
// holds the largest grid any compiled variant can use for this frame size.
size_t partials_capacity(const stpi_problem *p) {
    const DtypeOps *ops = ops_for(p->dtype);
    size_t cap = (size_t)NORM_BLOCKS_HOST;
    for (int i = 0; i < ops->nvariants; ++i) {
        const size_t g = (size_t)tiles_for(ops->variants[i], p) * STPI_NSEG_MAX;
        if (g > cap) cap = g;
    }
    for (int i = 0; i < ops->nadj; ++i) {
        const AdjVariant &v = ops->adj_variants[i];
        const size_t g = (size_t)(((p->W + v.TW - 1) / v.TW) * ((p->H + v.TH - 1) / v.TH)) * STPI_NSEG_MAX;
        if (g > cap) cap = g;
    }
    return cap;
}

WsLayout layout_for(const stpi_problem *p) {
    WsLayout L;
    const DtypeOps *ops = ops_for(p->dtype);
    const size_t N = (size_t)p->T * p->H * p->W;
    L.state_off = 0;
    L.partials_off = 256;
    L.partials_cap = partials_capacity(p);
    size_t off = L.partials_off + L.partials_cap * 2 * sizeof(double);
    off = (off + 255) & ~(size_t)255;
    L.buf_off = off;
    L.total = off + ((N * ops->elem + 255) & ~(size_t)255);
    return L;
}

static int g_forced_variant = -1;

// Captured iteration chains, keyed by every argument that shapes the launch
// sequence. Replaying a graph removes the per-launch host overhead of the
// 2 * max_iters + 3 kernels.
struct GraphKey {
    stpi_problem p;
    const void *f;
    void *x, *ws;
    int init, max_iters;
    double tol;
    const Variant *v;
    hipStream_t s;
    int part;   // ChainPart
    int pform;  // product-form chain
    bool operator==(const GraphKey &o) const {
        return std::memcmp(&p, &o.p, sizeof(p)) == 0 && f == o.f && x == o.x && ws == o.ws && init == o.init &&
               max_iters == o.max_iters && tol == o.tol && v == o.v && s == o.s && part == o.part &&
               pform == o.pform;
    }
};
struct GraphEntry {
    GraphKey key;
    hipGraphExec_t exec;
    hipEvent_t launched;  // recorded after every launch: eviction waits for it
    unsigned long long last_use;
};
static std::mutex g_graph_mu;
static std::vector<GraphEntry> g_graphs;
static unsigned long long g_graph_clock = 0;
constexpr size_t GRAPH_CACHE_MAX = 16;

// STPI_NO_FUSE=1 keeps the step finalisation in its own kernel (for comparison).
bool fusion_disabled() {
    const char *e = std::getenv("STPI_NO_FUSE");
    return e && e[0] == '1';
}

static bool graphs_enabled() {
    const char *e = std::getenv("STPI_NO_GRAPH");
    return !(e && e[0] == '1');
}

// Chains on a matrix-core variant run in product form (one staged array per
// step) unless STPI_NO_PRODUCT=1; a chain of no steps keeps the plain form.
int chain_pform(const Variant *v, int max_iters) {
    const char *e = std::getenv("STPI_NO_PRODUCT");
    return v && v->launch_p && max_iters > 0 && !(e && e[0] == '1') ? 1 : 0;
}

int forced_variant() { return g_forced_variant; }
void set_forced_variant(int v) { g_forced_variant = v; }

enum ChainPart { CHAIN_ALL = 0, CHAIN_HEAD = 1, CHAIN_CHUNK_PART = 2, CHAIN_TAIL = 3 };

struct ChainArgs {
    const stpi_problem *p;
    const DtypeOps *ops;
    const Variant *v;
    const void *f;
    void *x, *buf1;
    DevState *state;
    double *partials;
    int init, max_iters;
    double tol;
    int pform;
};

int enqueue_chain_part(const ChainArgs &a, int part, hipStream_t s) {
    switch (part) {
        case CHAIN_ALL:
            return enqueue_iteration(a.p, a.ops, a.v, a.f, a.x, a.buf1, a.state, a.partials, a.init, a.max_iters,
                                     a.tol, s, a.pform);
        case CHAIN_HEAD: {
            const int rc = enqueue_chain_init(a.p, a.ops, a.x, a.state, a.partials, a.init, a.max_iters, a.tol, s,
                                              a.v, a.f, a.buf1, a.pform);
            return rc ? rc
                      : enqueue_chain_steps(a.p, a.v, a.f, a.x, a.buf1, a.state, a.partials, CHAIN_CHUNK, s, a.pform);
        }
        case CHAIN_CHUNK_PART:
            return enqueue_chain_steps(a.p, a.v, a.f, a.x, a.buf1, a.state, a.partials, CHAIN_CHUNK, s, a.pform);
        default:
            return enqueue_chain_tail(a.p, a.ops, a.f, a.x, a.buf1, a.state, s, a.pform);
    }
}

// Launches the cached graph for key, capturing `enqueue` into a new one on a miss.
// A graph may still be queued when its entry is evicted (callers need not
// synchronise between calls), so every launch records the entry's event and
// eviction waits for it before destroying the executable graph.
template <class F>
int launch_cached_graph(const GraphKey &key, F &&enqueue, hipStream_t s) {
    hipGraphExec_t exec = nullptr;
    hipEvent_t launched = nullptr;
    hipError_t e;
    {
        std::lock_guard<std::mutex> lk(g_graph_mu);
        for (auto &g : g_graphs)
            if (g.key == key) {
                exec = g.exec;
                launched = g.launched;
                g.last_use = ++g_graph_clock;
                // launch under the lock: no other thread can evict the entry in between
                if ((e = hipGraphLaunch(exec, s)) != hipSuccess) return hip_fail(e, "graph launch");
                if ((e = hipEventRecord(launched, s)) != hipSuccess) return hip_fail(e, "graph event");
                return STPI_OK;
            }
    }
    if (!exec) {
        if ((e = hipStreamBeginCapture(s, hipStreamCaptureModeThreadLocal)) != hipSuccess)
            return hip_fail(e, "begin capture");
        const int rc = enqueue();
        hipGraph_t graph = nullptr;
        e = hipStreamEndCapture(s, &graph);
        if (rc) {
            if (graph) (void)hipGraphDestroy(graph);
            return rc;
        }
        if (e != hipSuccess) return hip_fail(e, "end capture");
        e = hipGraphInstantiate(&exec, graph, nullptr, nullptr, 0);
        (void)hipGraphDestroy(graph);
        if (e != hipSuccess) return hip_fail(e, "graph instantiate");
        if ((e = hipEventCreateWithFlags(&launched, hipEventDisableTiming)) != hipSuccess) {
            (void)hipGraphExecDestroy(exec);
            return hip_fail(e, "graph event");
        }
        std::lock_guard<std::mutex> lk(g_graph_mu);
        if (g_graphs.size() >= GRAPH_CACHE_MAX) {
            size_t old = 0;
            for (size_t i = 1; i < g_graphs.size(); ++i)
                if (g_graphs[i].last_use < g_graphs[old].last_use) old = i;
            (void)hipEventSynchronize(g_graphs[old].launched);
            (void)hipGraphExecDestroy(g_graphs[old].exec);
            (void)hipEventDestroy(g_graphs[old].launched);
            g_graphs.erase(g_graphs.begin() + old);
        }
        g_graphs.push_back(GraphEntry{key, exec, launched, ++g_graph_clock});
        if ((e = hipGraphLaunch(exec, s)) != hipSuccess) return hip_fail(e, "graph launch");
        if ((e = hipEventRecord(launched, s)) != hipSuccess) return hip_fail(e, "graph event");
    }
    return STPI_OK;
}

// Host-visible copy of the iteration state for the stop-flag poll (pinned,
// one per thread, kept for the life of the process), and its event.
DevState *pinned_state() {
    thread_local DevState *buf = nullptr;
    if (!buf && hipHostMalloc((void **)&buf, sizeof(DevState), hipHostMallocDefault) != hipSuccess) buf = nullptr;
    return buf;
}

hipEvent_t poll_event() {
    thread_local hipEvent_t ev = nullptr;
    if (!ev && hipEventCreateWithFlags(&ev, hipEventDisableTiming) != hipSuccess) ev = nullptr;
    return ev;
}

}  // namespace stpi

using namespace stpi;

extern "C" {

const char *stpi_status_string(int status) {
    switch (status) {
        case STPI_OK: return "ok";
        case STPI_EINVAL: return "invalid argument";
        case STPI_EUNSUPPORTED: return "unsupported problem";
        case STPI_EZERO_NORM: return "zero norm (A x = 0)";
        case STPI_ENONFINITE: return "non-finite value";
        case STPI_EHIP: return "HIP runtime error";
        case STPI_EWORKSPACE: return "workspace missing or too small";
        default: return "unknown status";
    }
}

const char *stpi_last_error(void) { return g_last_error.c_str(); }

const char *stpi_version(void) { return "stpi 0.1 gfx950"; }

size_t stpi_workspace_bytes(const stpi_problem *p) {
    if (validate_problem(p) != STPI_OK) return 0;
    return layout_for(p).total;
}

// Matrix-core variants scale their half-precision operands by a bound on
// |f x_stored| (times |x_scale|, applied in the kernel); it is computed here
// into the workspace's state area, which a single step does not otherwise use.
static hipError_t single_step_bound(const Variant *v, const stpi_problem *p, const void *f, const void *x, void *ws,
                                    FwdLaunch &FL, hipStream_t s) {
    if (v->PIPE != 3) return hipSuccess;
    uint32_t *w = &((DevState *)ws)->ubound;
    FL.ubound = w;
    hipError_t e = launch_clear_word(w, s);
    if (e == hipSuccess) e = ops_for(p->dtype)->bound((size_t)p->T * p->H * p->W, f, x, w, s);
    return e;
}

int stpi_step(const stpi_problem *p, const void *f, const void *x, double x_scale, void *z, double *d_sums,
              void *ws, size_t ws_bytes, void *stream) {
    clear_error();
    int rc = validate_problem(p);
    if (rc) return rc;
    if (!f || !x || !z || !d_sums) return fail(STPI_EINVAL, "NULL buffer");
    if (z == f || z == x) return fail(STPI_EINVAL, "z must not alias f or x");
    if (!std::isfinite(x_scale)) return fail(STPI_EINVAL, "x_scale must be finite");
    const WsLayout L = layout_for(p);
    if (!ws || ws_bytes < L.total) return fail(STPI_EWORKSPACE, "workspace needs %zu bytes", L.total);
    const Variant *v = choose_variant(p, forced_variant());
    if (!v) return fail(STPI_EUNSUPPORTED, "no compiled kernel for radii (%d, %d)", p->r_s, p->r_t);
    hipStream_t s = (hipStream_t)stream;
    FwdLaunch FL;
    std::memset(&FL, 0, sizeof(FL));
    FL.f = f;
    FL.buf0 = const_cast<void *>(x);
    FL.buf1 = z;
    FL.state = nullptr;
    FL.x_scale = x_scale;
    FL.partials = (double *)((char *)ws + L.partials_off);
    FL.T = p->T;
    FL.H = p->H;
    FL.W = p->W;
    FL.nseg = segments_for(*v, p);
    make_taps(p, FL.gs, FL.gt);
    hipError_t e = single_step_bound(v, p, f, x, ws, FL, s);
    if (e != hipSuccess) return hip_fail(e, "operand bound");
    e = v->launch(FL, s);
    if (e != hipSuccess) return hip_fail(e, "step kernel launch");
    e = launch_step_sums(FL.partials, grid_blocks(*v, p), x_scale, d_sums, s);
    if (e != hipSuccess) return hip_fail(e, "step sums launch");
    return STPI_OK;
}

}  // extern "C"

namespace stpi {

// Scratch of stpi_step_noalloc: the operand-bound word (first 256 bytes) and
// the step kernel's per-workgroup partial sums. Each device holds its own copy
// for the life of the process; host code reaches it only through the address
// hipGetSymbolAddress returns on that device (the array's name on the host is
// a stand-in, not a device address).
static __device__ __align__(256) unsigned char scratch[STPI_NOALLOC_SCRATCH_BYTES];

constexpr int MAX_DEVICES = 64;
static void *g_scratch_ptr[MAX_DEVICES];
static std::mutex g_scratch_mu;

// The scratch address on the current device (looked up once per device).
static int scratch_for_current_device(void **out) {
    int dev = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return hip_fail(e, "hipGetDevice");
    if (dev < 0 || dev >= MAX_DEVICES) return fail(STPI_EUNSUPPORTED, "device index %d out of range", dev);
    std::lock_guard<std::mutex> lk(g_scratch_mu);
    if (!g_scratch_ptr[dev]) {
        void *ptr = nullptr;
        e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
        if (e != hipSuccess) return hip_fail(e, "hipGetSymbolAddress(scratch)");
        if (!ptr) return fail(STPI_EHIP, "hipGetSymbolAddress(scratch) returned NULL");
        g_scratch_ptr[dev] = ptr;
    }
    *out = g_scratch_ptr[dev];
    return STPI_OK;
}

}  // namespace stpi

extern "C" {

size_t stpi_step_noalloc_scratch_bytes(const stpi_problem *p) {
    if (validate_problem(p) != STPI_OK) return 0;
    const Variant *v = choose_variant(p, forced_variant());
    if (!v) return 0;
    return 256 + (size_t)grid_blocks(*v, p) * 2 * sizeof(double);
}

int stpi_step_noalloc(const stpi_problem *p, const void *f, const void *x, double x_scale, void *z, double *d_sums,
                      void *stream) {
    clear_error();
    int rc = validate_problem(p);
    if (rc) return rc;
    if (!f || !x || !z || !d_sums) return fail(STPI_EINVAL, "NULL buffer");
    if (z == f || z == x) return fail(STPI_EINVAL, "z must not alias f or x");
    if (!std::isfinite(x_scale)) return fail(STPI_EINVAL, "x_scale must be finite");
    const Variant *v = choose_variant(p, forced_variant());
    if (!v) return fail(STPI_EUNSUPPORTED, "no compiled kernel for radii (%d, %d)", p->r_s, p->r_t);
    const int nunits = grid_blocks(*v, p);
    const size_t need = 256 + (size_t)nunits * 2 * sizeof(double);
    if (need > (size_t)STPI_NOALLOC_SCRATCH_BYTES)
        return fail(STPI_EUNSUPPORTED, "frame %dx%d needs %zu bytes of step scratch, above the %d-byte limit", p->H,
                    p->W, need, STPI_NOALLOC_SCRATCH_BYTES);
    void *scr = nullptr;
    if ((rc = scratch_for_current_device(&scr)) != STPI_OK) return rc;
    hipStream_t s = (hipStream_t)stream;
    FwdLaunch FL;
    std::memset(&FL, 0, sizeof(FL));
    FL.f = f;
    FL.buf0 = const_cast<void *>(x);
    FL.buf1 = z;
    FL.state = nullptr;
    FL.x_scale = x_scale;
    FL.partials = (double *)((char *)scr + 256);
    FL.T = p->T;
    FL.H = p->H;
    FL.W = p->W;
    FL.nseg = segments_for(*v, p);
    make_taps(p, FL.gs, FL.gt);
    hipError_t e = hipSuccess;
    if (v->PIPE == 3) {
        // the bound word is cleared by a kernel and raised by the bound pass
        uint32_t *w = (uint32_t *)scr;
        FL.ubound = w;
        e = launch_clear_word(w, s);
        if (e == hipSuccess) e = ops_for(p->dtype)->bound((size_t)p->T * p->H * p->W, f, x, w, s);
        if (e != hipSuccess) return hip_fail(e, "operand bound");
    }
    e = v->launch(FL, s);
    if (e != hipSuccess) return hip_fail(e, "step kernel launch");
    e = launch_step_sums(FL.partials, nunits, x_scale, d_sums, s);
    if (e != hipSuccess) return hip_fail(e, "step sums launch");
    return STPI_OK;
}

int stpi_iterate(const stpi_problem *p, const void *f, void *x, int init, int max_iters, double tol, void *ws,
                 size_t ws_bytes, stpi_result *out, void *stream) {
    clear_error();
    int rc = validate_problem(p);
    if (rc) return rc;
    if (!f || !x) return fail(STPI_EINVAL, "NULL buffer");
    if (f == x) return fail(STPI_EINVAL, "x must not alias f");
    if (max_iters < 0) return fail(STPI_EINVAL, "max_iters must be >= 0");
    if (init < 0 || init > 2) return fail(STPI_EINVAL, "init must be 0 (use x), 1 (uniform) or 2 (use x, rise check)");
    if (!std::isfinite(tol)) return fail(STPI_EINVAL, "tol must be finite");
    const WsLayout L = layout_for(p);
    if (!ws || ws_bytes < L.total) return fail(STPI_EWORKSPACE, "workspace needs %zu bytes", L.total);
    const Variant *v = choose_variant(p, forced_variant());
    if (!v) return fail(STPI_EUNSUPPORTED, "no compiled kernel for radii (%d, %d)", p->r_s, p->r_t);
    if (out) std::memset(out, 0, sizeof(*out));
    hipStream_t s = (hipStream_t)stream;
    const DtypeOps *ops = ops_for(p->dtype);
    const size_t N = (size_t)p->T * p->H * p->W;
    DevState *state = (DevState *)((char *)ws + L.state_off);
    double *partials = (double *)((char *)ws + L.partials_off);
    void *buf1 = (char *)ws + L.buf_off;

    // A run in tolerance mode stops early, but a chain of max_iters steps
    // would still launch every (step, finalise) pair (they exit at once when
    // done, at a launch latency each). Long tolerance runs therefore replay a
    // chain of CHAIN_CHUNK steps, the host checking the stop flag one chunk
    // behind so the device never waits for it.
    const bool chunked = tol > 0.0 && max_iters > 2 * CHAIN_CHUNK;
    const int pform = chain_pform(v, max_iters);
    ChainArgs ca{p, ops, v, f, x, buf1, state, partials, init, max_iters, tol, pform};
    const bool use_graphs = s != nullptr && graphs_enabled();
    auto run = [&](int part) -> int {
        if (!use_graphs) return enqueue_chain_part(ca, part, s);
        GraphKey key;
        std::memset(&key, 0, sizeof(key));
        key.p = *p;
        key.f = f;
        key.x = x;
        key.ws = ws;
        key.init = init;
        key.max_iters = max_iters;
        key.tol = tol;
        key.v = v;
        key.s = s;
        key.part = part;
        key.pform = pform;
        return launch_cached_graph(key, [&] { return enqueue_chain_part(ca, part, s); }, s);
    };
    if (!chunked) {
        if ((rc = run(CHAIN_ALL))) return rc;
    } else {
        if ((rc = run(CHAIN_HEAD))) return rc;
        DevState *poll = pinned_state();
        hipEvent_t ev = poll_event();
        if (!poll || !ev) return fail(STPI_EHIP, "pinned poll buffer or event unavailable");
        hipError_t e;
        for (int issued = CHAIN_CHUNK; issued < max_iters; issued += CHAIN_CHUNK) {
            // state after the chunks issued so far, then one more chunk while it travels
            if ((e = hipMemcpyAsync(poll, state, sizeof(DevState), hipMemcpyDeviceToHost, s)) != hipSuccess)
                return hip_fail(e, "state poll");
            if ((e = hipEventRecord(ev, s)) != hipSuccess) return hip_fail(e, "poll event");
            if ((rc = run(CHAIN_CHUNK_PART))) return rc;
            if ((e = hipEventSynchronize(ev)) != hipSuccess) return hip_fail(e, "poll wait");
            if (poll->done) break;
        }
        if ((rc = run(CHAIN_TAIL))) return rc;
    }
    if (!out) return STPI_OK;

    DevState hs;
    hipError_t e = hipMemcpyAsync(&hs, state, sizeof(hs), hipMemcpyDeviceToHost, s);
    if (e != hipSuccess) return hip_fail(e, "state readback");
    e = hipStreamSynchronize(s);
    if (e != hipSuccess) return hip_fail(e, "stream synchronize");
    out->iters = hs.iters;
    out->converged = hs.converged;
    out->flags = hs.flags;
    out->residual = hs.residual;
    out->lambda = hs.lambda;
    out->rayleigh = hs.rayleigh;
    out->first_residuals[0] = hs.first_res[0];
    out->first_residuals[1] = hs.first_res[1];
    out->status = STPI_OK;
    if (hs.flags & FLAG_SYNC) {
        out->status = STPI_EHIP;
        return fail(STPI_EHIP, "a step's partial sums did not arrive (step %d)", hs.iters + 1);
    }
    if (hs.flags & FLAG_NONFINITE) out->status = STPI_ENONFINITE;
    else if (hs.flags & FLAG_ZERO) out->status = STPI_EZERO_NORM;
    (void)N;
    if (out->status != STPI_OK)
        return fail(out->status, "iteration stopped after %d steps: %s", hs.iters, stpi_status_string(out->status));
    return STPI_OK;
}

int stpi_time_step(const stpi_problem *p, const void *f, const void *x, void *z, void *ws, size_t ws_bytes,
                   int variant, int reps, void *stream, double *avg_ms) {
    clear_error();
    int rc = validate_problem(p);
    if (rc) return rc;
    if (!f || !x || !z || !avg_ms) return fail(STPI_EINVAL, "NULL buffer");
    if (reps < 1) return fail(STPI_EINVAL, "reps must be >= 1");
    const WsLayout L = layout_for(p);
    if (!ws || ws_bytes < L.total) return fail(STPI_EWORKSPACE, "workspace needs %zu bytes", L.total);
    const Variant *v = choose_variant(p, variant >= 0 ? variant : forced_variant());
    if (!v) return fail(STPI_EUNSUPPORTED, "no eligible kernel variant");
    hipStream_t s = (hipStream_t)stream;
    FwdLaunch FL;
    std::memset(&FL, 0, sizeof(FL));
    FL.f = f;
    FL.buf0 = const_cast<void *>(x);
    FL.buf1 = z;
    FL.x_scale = 1.0;
    FL.partials = (double *)((char *)ws + L.partials_off);
    FL.T = p->T;
    FL.H = p->H;
    FL.W = p->W;
    FL.nseg = segments_for(*v, p);
    make_taps(p, FL.gs, FL.gt);
    hipEvent_t e0, e1;
    hipError_t e;
    if ((e = single_step_bound(v, p, f, x, ws, FL, s)) != hipSuccess) return hip_fail(e, "operand bound");
    if ((e = hipEventCreate(&e0)) != hipSuccess) return hip_fail(e, "event create");
    if ((e = hipEventCreate(&e1)) != hipSuccess) {
        (void)hipEventDestroy(e0);
        return hip_fail(e, "event create");
    }
    e = hipEventRecord(e0, s);
    for (int i = 0; i < reps && e == hipSuccess; ++i) e = v->launch(FL, s);
    if (e == hipSuccess) e = hipEventRecord(e1, s);
    if (e == hipSuccess) e = hipEventSynchronize(e1);
    float ms = 0.0f;
    if (e == hipSuccess) e = hipEventElapsedTime(&ms, e0, e1);
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    if (e != hipSuccess) return hip_fail(e, "timed launches");
    *avg_ms = (double)ms / reps;
    return STPI_OK;
}

int stpi_time_chain_step(const stpi_problem *p, const void *f, void *x, void *ws, size_t ws_bytes, int variant,
                         int reps, void *stream, double *avg_ms, int *product_form) {
    clear_error();
    int rc = validate_problem(p);
    if (rc) return rc;
    if (!f || !x || !avg_ms) return fail(STPI_EINVAL, "NULL buffer");
    if (f == x) return fail(STPI_EINVAL, "x must not alias f");
    if (reps < 1) return fail(STPI_EINVAL, "reps must be >= 1");
    const WsLayout L = layout_for(p);
    if (!ws || ws_bytes < L.total) return fail(STPI_EWORKSPACE, "workspace needs %zu bytes", L.total);
    const Variant *v = choose_variant(p, variant >= 0 ? variant : forced_variant());
    if (!v) return fail(STPI_EUNSUPPORTED, "no eligible kernel variant");
    hipStream_t s = (hipStream_t)stream;
    const DtypeOps *ops = ops_for(p->dtype);
    DevState *state = (DevState *)((char *)ws + L.state_off);
    double *partials = (double *)((char *)ws + L.partials_off);
    void *buf1 = (char *)ws + L.buf_off;
    // a fixed-count chain long enough that no timed step finds it done
    const int total = reps + 2;
    const int pform = chain_pform(v, total);
    if (product_form) *product_form = pform;
    rc = enqueue_chain_init(p, ops, x, state, partials, 1, total, 0.0, s, v, f, buf1, pform);
    // the steps as a fixed-count chain of `total` steps runs them
    if (!rc) rc = enqueue_chain_steps(p, v, f, x, buf1, state, partials, 1, s, pform, total, 0);
    if (rc) return rc;
    hipEvent_t e0, e1;
    hipError_t e;
    if ((e = hipEventCreate(&e0)) != hipSuccess) return hip_fail(e, "event create");
    if ((e = hipEventCreate(&e1)) != hipSuccess) {
        (void)hipEventDestroy(e0);
        return hip_fail(e, "event create");
    }
    e = hipEventRecord(e0, s);
    if (e == hipSuccess) rc = enqueue_chain_steps(p, v, f, x, buf1, state, partials, reps, s, pform, total, 1);
    if (e == hipSuccess && !rc) e = hipEventRecord(e1, s);
    if (e == hipSuccess && !rc) e = hipEventSynchronize(e1);
    float ms = 0.0f;
    if (e == hipSuccess && !rc) e = hipEventElapsedTime(&ms, e0, e1);
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    if (rc) return rc;
    if (e != hipSuccess) return hip_fail(e, "timed launches");
    *avg_ms = (double)ms / reps;
    return STPI_OK;
}

int stpi_variant_count(int dtype) {
    const DtypeOps *ops = ops_for(dtype);
    return ops ? ops->nvariants : 0;
}

int stpi_variant_info(int dtype, int index, int32_t info[9]) {
    clear_error();
    const DtypeOps *ops = ops_for(dtype);
    if (!ops || !info || index < 0 || index >= ops->nvariants)
        return fail(STPI_EINVAL, "no variant %d for dtype %d", index, dtype);
    const Variant &v = ops->variants[index];
    info[0] = v.RS;
    info[1] = v.RT;
    info[2] = v.TH;
    info[3] = v.TW;
    info[4] = v.NTHR;
    info[5] = v.RY;
    info[6] = v.QX;
    info[7] = v.OCC;
    info[8] = v.PIPE;
    return STPI_OK;
}

int stpi_launch_shape(const stpi_problem *p, int variant, int32_t info[5]) {
    clear_error();
    int rc = validate_problem(p);
    if (rc) return rc;
    if (!info) return fail(STPI_EINVAL, "NULL info");
    const DtypeOps *ops = ops_for(p->dtype);
    const Variant *v = choose_variant(p, variant >= 0 ? variant : forced_variant());
    if (!v) return fail(STPI_EUNSUPPORTED, "no compiled kernel for radii (%d, %d)", p->r_s, p->r_t);
    const int nseg = segments_for(*v, p);
    info[0] = (int32_t)(v - ops->variants);
    info[1] = grid_blocks(*v, p) / nseg;
    info[2] = nseg;
    info[3] = v->blocks_per_cu();
    info[4] = grid_blocks(*v, p);
    return STPI_OK;
}

int stpi_set_variant(int index) {
    clear_error();
    if (index < -1) return fail(STPI_EINVAL, "variant index must be >= -1");
    set_forced_variant(index);
    return STPI_OK;
}

}  // extern "C"

namespace stpi {

// Enqueues start vector, max_iters (step, finalise) pairs and the final
// normalisation. No host synchronisation.
int enqueue_chain_init(const stpi_problem *p, const DtypeOps *ops, void *x, DevState *state, double *partials,
                       int init, int max_iters, double tol, hipStream_t s, const Variant *v, const void *f,
                       void *buf1, int pform) {
    const size_t N = (size_t)p->T * p->H * p->W;
    hipError_t e;
    if (init == 1) {
        // product form: the first step stages f itself, the constant start is never stored
        if (!pform && (e = ops->fill_ones(x, N, s)) != hipSuccess) return hip_fail(e, "fill");
        if ((e = launch_state_init(state, 1.0 / std::sqrt((double)N), tol, max_iters, 0, pform ? 2 : 0, s)) !=
            hipSuccess)
            return hip_fail(e, "init");
    } else {
        if ((e = launch_state_init(state, 1.0, tol, max_iters, init == 2 ? 1 : 0, 0, s)) != hipSuccess)
            return hip_fail(e, "init");
        if ((e = ops->sumsq(x, N, partials, s)) != hipSuccess) return hip_fail(e, "norm");
        if ((e = launch_state_from_norm(partials, NORM_BLOCKS_HOST, state, s)) != hipSuccess)
            return hip_fail(e, "init norm");
    }
    // matrix-core steps scale their operands by max |f| (the iterate is unit)
    if (v && v->PIPE == 3 && (e = ops->bound(N, f, nullptr, &state->ubound, s)) != hipSuccess)
        return hip_fail(e, "operand bound");
    if (pform && init != 1 && (e = ops->to_product(f, x, buf1, N, state, s)) != hipSuccess)
        return hip_fail(e, "product-form start");
    // steps that finalise themselves poll their partial-sum slots
    if (v && (e = launch_partials_empty(partials, grid_blocks(*v, p), s)) != hipSuccess)
        return hip_fail(e, "partials");
    if ((e = hipGetLastError()) != hipSuccess) return hip_fail(e, "init");
    return STPI_OK;
}

int enqueue_chain_tail(const stpi_problem *p, const DtypeOps *ops, const void *f, void *x, void *buf1,
                       DevState *state, hipStream_t s, int pform) {
    const size_t N = (size_t)p->T * p->H * p->W;
    const hipError_t e =
        pform ? ops->from_product(x, buf1, f, N, state, s) : ops->normalize(x, buf1, N, state, s);
    return e == hipSuccess ? STPI_OK : hip_fail(e, "normalize");
}

int enqueue_chain_steps(const stpi_problem *p, const Variant *v, const void *f, void *x, void *buf1, DevState *state,
                        double *partials, int steps, hipStream_t s, int pform, int fixed_total, int k0) {
    hipError_t e;
    FwdLaunch FL;
    std::memset(&FL, 0, sizeof(FL));
    FL.f = f;
    FL.buf0 = x;
    FL.buf1 = buf1;
    FL.state = state;
    FL.ubound = &state->ubound;
    FL.partials = partials;
    FL.T = p->T;
    FL.H = p->H;
    FL.W = p->W;
    FL.nseg = segments_for(*v, p);
    make_taps(p, FL.gs, FL.gt);
    const int nb = grid_blocks(*v, p);
    // workgroups of FINAL_THREADS or more finalise the step themselves (the
    // last one to finish), saving a launch per step
    FL.fuse = v->NTHR >= FINAL_THREADS && !fusion_disabled() ? 1 : 0;
    const FwdLaunchFn launch = pform ? v->launch_p : v->launch;
    if (!launch) return fail(STPI_EUNSUPPORTED, "variant has no product-form step");
    for (int k = 0; k < steps; ++k) {
        const int kk = k0 + k;
        FL.no_prev = fixed_total > 0 && kk >= 2 && kk < fixed_total - 1 ? 1 : 0;
        if ((e = launch(FL, s)) != hipSuccess) return hip_fail(e, "step kernel launch");
        if (!FL.fuse && (e = launch_finalize(partials, nb, state, s)) != hipSuccess)
            return hip_fail(e, "finalize launch");
    }
    return STPI_OK;
}

int enqueue_iteration(const stpi_problem *p, const DtypeOps *ops, const Variant *v, const void *f, void *x,
                      void *buf1, DevState *state, double *partials, int init, int max_iters, double tol,
                      hipStream_t s, int pform) {
    int rc = enqueue_chain_init(p, ops, x, state, partials, init, max_iters, tol, s, v, f, buf1, pform);
    if (!rc) rc = enqueue_chain_steps(p, v, f, x, buf1, state, partials, max_iters, s, pform, tol > 0.0 ? 0 : max_iters);
    return rc ? rc : enqueue_chain_tail(p, ops, f, x, buf1, state, s, pform);
}

}  // namespace stpi
