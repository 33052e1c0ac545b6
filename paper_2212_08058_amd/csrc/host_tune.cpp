// Tile autotuner: times every compiled step variant that fits a problem with
// HIP events, keeps the fastest per (device arch, dtype, radii, frame size),
// and persists the table as text so later processes start tuned.
#include <hip/hip_runtime.h>

#include <cstdio>
#include <cstring>
#include <mutex>
#include <string>
#include <vector>

#include "../../include/stpi.h"
#include "host_internal.hpp"

namespace stpi {

struct TuneEntry {
    std::string arch;
    int dtype, rs, rt, H, W;
    int sig[9];  // RS, RT, TH, TW, NTHR, RY, QX, OCC, PIPE of the winner
    double ms;
};

static std::mutex g_tune_mu;
static std::vector<TuneEntry> g_tune;

static std::string device_arch() {
    int dev = 0;
    hipDeviceProp_t prop;
    if (hipGetDevice(&dev) != hipSuccess || hipGetDeviceProperties(&prop, dev) != hipSuccess) return "unknown";
    std::string a = prop.gcnArchName;
    const size_t colon = a.find(':');
    return colon == std::string::npos ? a : a.substr(0, colon);
}

static int variant_by_sig(int dtype, const int *sig) {
    const DtypeOps *ops = ops_for(dtype);
    if (!ops) return -1;
    for (int i = 0; i < ops->nvariants; ++i) {
        const Variant &v = ops->variants[i];
        const int s[9] = {v.RS, v.RT, v.TH, v.TW, v.NTHR, v.RY, v.QX, v.OCC, v.PIPE};
        if (std::memcmp(s, sig, sizeof(s)) == 0) return i;
    }
    return -1;
}

int tuned_variant(const stpi_problem *p) {
    std::lock_guard<std::mutex> lk(g_tune_mu);
    if (g_tune.empty()) return -1;
    const std::string arch = device_arch();
    for (const auto &e : g_tune)
        if (e.arch == arch && e.dtype == p->dtype && e.rs == p->r_s && e.rt == p->r_t && e.H == p->H && e.W == p->W)
            return variant_by_sig(p->dtype, e.sig);
    return -1;
}

static void put_entry(const TuneEntry &n) {
    for (auto &e : g_tune)
        if (e.arch == n.arch && e.dtype == n.dtype && e.rs == n.rs && e.rt == n.rt && e.H == n.H && e.W == n.W) {
            e = n;
            return;
        }
    g_tune.push_back(n);
}

static int save_table(const char *path) {
    const std::string tmp = std::string(path) + ".tmp";
    FILE *fp = std::fopen(tmp.c_str(), "w");
    if (!fp) return fail(STPI_EINVAL, "cannot write %s", tmp.c_str());
    std::fprintf(fp, "# stpi autotune v2: arch dtype r_s r_t H W RS RT TH TW NTHR RY QX OCC PIPE ms\n");
    for (const auto &e : g_tune)
        std::fprintf(fp, "%s %d %d %d %d %d %d %d %d %d %d %d %d %d %d %.6f\n", e.arch.c_str(), e.dtype, e.rs, e.rt,
                     e.H, e.W, e.sig[0], e.sig[1], e.sig[2], e.sig[3], e.sig[4], e.sig[5], e.sig[6], e.sig[7], e.sig[8],
                     e.ms);
    std::fclose(fp);
    if (std::rename(tmp.c_str(), path) != 0) return fail(STPI_EINVAL, "cannot rename %s", tmp.c_str());
    return STPI_OK;
}

}  // namespace stpi

using namespace stpi;

extern "C" {

int stpi_autotune_load(const char *path) {
    clear_error();
    if (!path) return fail(STPI_EINVAL, "NULL path");
    FILE *fp = std::fopen(path, "r");
    if (!fp) return fail(STPI_EINVAL, "cannot read %s", path);
    char line[512];
    int n = 0;
    std::lock_guard<std::mutex> lk(g_tune_mu);
    while (std::fgets(line, sizeof(line), fp)) {
        if (line[0] == '#') continue;
        char arch[64];
        TuneEntry e;
        if (std::sscanf(line, "%63s %d %d %d %d %d %d %d %d %d %d %d %d %d %d %lf", arch, &e.dtype, &e.rs, &e.rt,
                        &e.H, &e.W, &e.sig[0], &e.sig[1], &e.sig[2], &e.sig[3], &e.sig[4], &e.sig[5], &e.sig[6],
                        &e.sig[7], &e.sig[8], &e.ms) != 16)
            continue;
        e.arch = arch;
        put_entry(e);
        ++n;
    }
    std::fclose(fp);
    return STPI_OK;
}

void stpi_autotune_clear(void) {
    std::lock_guard<std::mutex> lk(g_tune_mu);
    g_tune.clear();
}

int stpi_autotune(const stpi_problem *p, const char *cache_path, int reps, int32_t *best_variant, double *best_ms) {
    clear_error();
    int rc = validate_problem(p);
    if (rc) return rc;
    if (reps < 1) return fail(STPI_EINVAL, "reps must be >= 1");
    const DtypeOps *ops = ops_for(p->dtype);
    const size_t N = (size_t)p->T * p->H * p->W;
    const size_t bytes = N * ops->elem;
    const size_t wsb = stpi_workspace_bytes(p);
    void *f = nullptr, *x = nullptr, *ws = nullptr;
    hipError_t e = hipMalloc(&f, bytes);
    if (e == hipSuccess) e = hipMalloc(&x, bytes);
    if (e == hipSuccess) e = hipMalloc(&ws, wsb);
    if (e == hipSuccess) e = ops->fill_ones(f, N, nullptr);
    if (e == hipSuccess) e = hipDeviceSynchronize();
    int best = -1;
    double best_t = 1e300;
    if (e == hipSuccess) {
        // each variant as an iteration chain runs it (its product form where it has one)
        for (int i = 0; i < ops->nvariants && rc == STPI_OK; ++i) {
            const Variant &v = ops->variants[i];
            if (v.RS < p->r_s || v.RT < p->r_t) continue;
            double ms = 0.0;
            rc = stpi_time_chain_step(p, f, x, ws, wsb, i, 1, nullptr, &ms, nullptr);  // warm-up
            if (rc == STPI_OK) rc = stpi_time_chain_step(p, f, x, ws, wsb, i, reps, nullptr, &ms, nullptr);
            if (rc == STPI_OK && ms < best_t) {
                best_t = ms;
                best = i;
            }
        }
    }
    if (f) (void)hipFree(f);
    if (x) (void)hipFree(x);
    if (ws) (void)hipFree(ws);
    if (e != hipSuccess) return hip_fail(e, "autotune buffers");
    if (rc) return rc;
    if (best < 0) return fail(STPI_EUNSUPPORTED, "no compiled kernel for radii (%d, %d)", p->r_s, p->r_t);
    const Variant &v = ops->variants[best];
    TuneEntry te;
    te.arch = device_arch();
    te.dtype = p->dtype;
    te.rs = p->r_s;
    te.rt = p->r_t;
    te.H = p->H;
    te.W = p->W;
    const int sig[9] = {v.RS, v.RT, v.TH, v.TW, v.NTHR, v.RY, v.QX, v.OCC, v.PIPE};
    std::memcpy(te.sig, sig, sizeof(sig));
    te.ms = best_t;
    {
        std::lock_guard<std::mutex> lk(g_tune_mu);
        put_entry(te);
        if (cache_path && (rc = save_table(cache_path))) return rc;
    }
    if (best_variant) *best_variant = best;
    if (best_ms) *best_ms = best_t;
    return STPI_OK;
}

}  // extern "C"
