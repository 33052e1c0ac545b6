// Declarations shared by the host-side translation units of libstpi.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdarg>
#include <cstddef>

#include "../../include/stpi.h"
#include "common.hpp"
#include "batch.hpp"
#include "dtype_ops.hpp"

namespace stpi {

constexpr int NORM_BLOCKS_HOST = 512;  // grid of the sum-of-squares pass (matches NORM_BLOCKS)

struct WsLayout {
    size_t state_off, partials_off, partials_cap, buf_off, total;
};

int fail(int status, const char *fmt, ...);
int hip_fail(hipError_t e, const char *where);
void clear_error();
const DtypeOps *ops_for(int dtype);
int validate_problem(const stpi_problem *p);
void make_taps(const stpi_problem *p, double *gs, double *gt);
// allow_mfma false skips the matrix-core variants (callers that cannot supply
// their operand bound).
const Variant *choose_variant(const stpi_problem *p, int forced_index, bool allow_mfma = true);
int grid_blocks(const Variant &v, const stpi_problem *p);
int segments_for(const Variant &v, const stpi_problem *p);
// Phases of the slowest of k frame segments of a T-frame tile, and the split
// of a tile the occupancy rules leave whole (see host.cpp).
int segment_phases(int T, int RT, int k);
int split_short_tiles(int tiles, int T, int RT);
constexpr int STPI_NSEG_MAX = 8;  // frame segments per tile at most
WsLayout layout_for(const stpi_problem *p);
constexpr int CHAIN_CHUNK = 16;  // steps per replayed chain segment in long tolerance runs
// pform: run the chain in product form (chain_pform decides).
int chain_pform(const Variant *v, int max_iters);
int enqueue_chain_init(const stpi_problem *p, const DtypeOps *ops, void *x, DevState *state, double *partials,
                       int init, int max_iters, double tol, hipStream_t s, const Variant *v, const void *f,
                       void *buf1, int pform);
// fixed_total > 0: the steps are steps k0 .. k0 + steps - 1 of a chain of
// fixed_total steps with no tolerance, whose inner products with the
// previous iterate (residual, Rayleigh quotient) are used only on the first
// two steps and the last: the others do not read the previous iterate.
int enqueue_chain_steps(const stpi_problem *p, const Variant *v, const void *f, void *x, void *buf1, DevState *state,
                        double *partials, int steps, hipStream_t s, int pform, int fixed_total = 0, int k0 = 0);
int enqueue_chain_tail(const stpi_problem *p, const DtypeOps *ops, const void *f, void *x, void *buf1,
                       DevState *state, hipStream_t s, int pform);
int enqueue_iteration(const stpi_problem *p, const DtypeOps *ops, const Variant *v, const void *f, void *x,
                      void *buf1, DevState *state, double *partials, int init, int max_iters, double tol,
                      hipStream_t s, int pform);

// Variant selection overrides (autotuner and tests).
int forced_variant();
int tuned_variant(const stpi_problem *p);

hipError_t launch_state_init(DevState *s, double scale, double tol, int max_iters, int check_rise, int pform,
                             hipStream_t st);
hipError_t launch_state_from_norm(const double *partials, int n, DevState *s, hipStream_t st);
hipError_t launch_clear_word(uint32_t *w, hipStream_t st);
hipError_t launch_partials_empty(double *partials, int n, hipStream_t st);
bool fusion_disabled();
int device_cus();  // compute units of the current device
hipError_t launch_finalize(const double *partials, int n, DevState *s, hipStream_t st);
hipError_t launch_step_sums(const double *partials, int n, double x_scale, double *d_sums, hipStream_t st);
hipError_t launch_combine_bwd_finalize(int C, int nblocks, const double *partials, const double *w, double *gw,
                                       hipStream_t st);
hipError_t launch_max_finalize(int nblocks, const double *partials, double *scalars, hipStream_t st);
hipError_t launch_dot_finalize(const double *partials, int n, const double *a_norm, double *out, hipStream_t st);
hipError_t launch_norm_finalize(const double *partials, int n, double *out, hipStream_t st);
hipError_t launch_sum0_finalize(const double *partials, int n, double *out, hipStream_t st);
hipError_t launch_batch_init(DevState *states, const ClipDesc *clips, int nclips, double tol, int max_iters,
                             int uniform, int check_rise, int pform, BatchCtl *ctl, hipStream_t st);
hipError_t launch_batch_compact(const DevState *states, const ClipDesc *clips, const int32_t *clip_order, int nclips,
                                int32_t *active_clip, int32_t *active_cum, BatchCtl *ctl, hipStream_t st);
hipError_t launch_batch_state_from_norm(const double *partials, DevState *states, int nclips, BatchCtl *ctl,
                                        hipStream_t st);
hipError_t launch_batch_finalize(const double *partials, const ClipDesc *clips, DevState *states, int nclips,
                                 BatchCtl *ctl, hipStream_t st);
hipError_t launch_adamw(int dtype, int64_t n, void *w, const void *g, void *m, void *v, void *vmax, double lr,
                        double beta1, double beta2, double eps, double wd, double bc1, double bc2, int amsgrad,
                        hipStream_t st);

}  // namespace stpi
