/*
 * stpi: space-time power iteration on MI355X (gfx950).
 *
 * C ABI of the library libstpi.so. The library computes the principal
 * eigenvector of the pixel-level space-time affinity matrix
 *
 *     A = diag(f) G diag(f),
 *     G_ij = exp(-dt^2/(2 sigma_t^2) - (dy^2 + dx^2)/(2 sigma_s^2))
 *            for |dt| <= r_t, |dy| <= r_s, |dx| <= r_s, both voxels inside
 *            the T x H x W volume (zero padding), 0 otherwise,
 *
 * by matrix-free power iteration x <- A x / ||A x||_2. This is the paper's
 * Gaussian affinity in its first-order form (Sec. 3, Eq. 2) with alpha = 0 and
 * the unary feature taken as f; the neighbourhood sum of Eq. 4 is evaluated as
 * the first 3D convolution term of Eq. 7, split into three 1D passes (the
 * separable filter of Sec. 4, "Computational complexity"), followed by the global L2 normalisation of
 * Eq. 8. The kernel is not normalised: G_ii = 1.
 *
 * Conventions for every entry point:
 *  - Volumes are dense row-major [T][H][W] (W fastest) arrays in DEVICE
 *    memory, element type given by stpi_problem.dtype. Batched inputs are
 *    one flat device buffer addressed by per-clip element offsets.
 *  - The caller owns every buffer and the stream; the library allocates
 *    nothing on the hot path. `stream` is a hipStream_t passed as void*
 *    (NULL = the default stream). Calls are asynchronous on that stream
 *    unless stated otherwise.
 *  - Arguments are validated on the host before any launch; on error
 *    nothing is written and a status code is returned. The message of the
 *    last error on the calling thread is available from stpi_last_error().
 *  - f must be finite and >= 0 for Perron semantics (not checked on the
 *    hot path).
 */
#ifndef STPI_H
#define STPI_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* ---- status codes -------------------------------------------------------- */
#define STPI_OK 0
#define STPI_EINVAL 1        /* bad argument (checked before any launch)          */
#define STPI_EUNSUPPORTED 2  /* valid but outside the compiled kernel set         */
#define STPI_EZERO_NORM 3    /* A x = 0 (e.g. f == 0); x keeps the last iterate   */
#define STPI_ENONFINITE 4    /* a NaN or Inf appeared in a norm                    */
#define STPI_EHIP 5          /* HIP runtime error; see stpi_last_error()          */
#define STPI_EWORKSPACE 6    /* workspace missing or too small                    */

/* Radius limits of the compiled kernels. */
#define STPI_MAX_RS 16
#define STPI_MAX_RT 8

/* ---- element types ------------------------------------------------------- */
#define STPI_F32 0   /* float storage, float arithmetic                          */
#define STPI_BF16 1  /* bfloat16 storage (RNE on store), float arithmetic        */
#define STPI_F64 2   /* double storage and arithmetic (gradient checks)          */

/* One clip and its filter. T, H, W >= 1; sigma_s, sigma_t > 0;
 * 0 <= r_s <= STPI_MAX_RS; 0 <= r_t <= STPI_MAX_RT. */
typedef struct stpi_problem {
    int32_t T, H, W;
    float sigma_s, sigma_t;
    int32_t r_s, r_t;
    int32_t dtype;
} stpi_problem;

/* Outcome of an iteration (host memory). residual is ||x_k - x_{k-1}||_2
 * between the last two unit iterates; lambda = ||A x_{k-1}|| (tends to the
 * principal eigenvalue); rayleigh = <x_{k-1}, A x_{k-1}>. flags: bit 0 zero
 * norm, bit 1 non-finite, bit 2 stopped by the init = 2 rise check. Not
 * converging is not an error (converged = 0).
 * first_residuals: the residuals after the first and second applications of
 * this call (0 where not reached), e.g. for a warm start's fallback rule. */
typedef struct stpi_result {
    int32_t iters;
    int32_t converged;
    uint32_t flags;
    int32_t status;
    double residual;
    double lambda;
    double rayleigh;
    double first_residuals[2];
} stpi_result;

/* Message for a status code; never NULL. */
const char *stpi_status_string(int status);
/* Message of the last error on the calling thread ("" if none). */
const char *stpi_last_error(void);
/* Library version string. */
const char *stpi_version(void);

/* Bytes of device workspace stpi_iterate / stpi_step need for `p` (includes
 * one volume-sized ping-pong buffer, block partials and the iteration state).
 * Returns 0 if `p` is invalid. */
size_t stpi_workspace_bytes(const stpi_problem *p);

/* One application of A (Eq. 4 / Eq. 7 first term), unnormalised:
 *   z = f .* G * (f .* (x * x_scale)),
 *   d_sums[0] = sum z^2,  d_sums[1] = sum z .* x * x_scale   (device doubles).
 * f, x, z: device volumes of p->dtype; z must not alias f or x. d_sums: two
 * device doubles. ws: workspace of stpi_workspace_bytes(p). */
int stpi_step(const stpi_problem *p, const void *f, const void *x, double x_scale, void *z,
              double *d_sums, void *ws, size_t ws_bytes, void *stream);

/* For callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc): stpi_step
 * without a workspace argument. Same arguments, results and errors as
 * stpi_step; the block partial sums and the operand-bound word live in a
 * library-owned device array of STPI_NOALLOC_SCRATCH_BYTES per GPU, held
 * until the process ends. The call allocates nothing (no hipMalloc, no
 * library allocation). Problems whose launch needs more scratch than that
 * (stpi_step_noalloc_scratch_bytes(p) > STPI_NOALLOC_SCRATCH_BYTES, frames
 * of tens of millions of pixels) get STPI_EUNSUPPORTED before any launch.
 * Every call on one GPU shares that GPU's array: calls that overlap on one
 * device (different streams, or host threads without ordering) race and
 * must be serialised by the caller. The array keeps the last call's
 * contents; the call clears what must start at zero itself. */
#define STPI_NOALLOC_SCRATCH_BYTES (1 << 20)
size_t stpi_step_noalloc_scratch_bytes(const stpi_problem *p);
int stpi_step_noalloc(const stpi_problem *p, const void *f, const void *x, double x_scale, void *z,
                      double *d_sums, void *stream);

/* Power iteration (Eq. 4 + Eq. 8, outer loop of Alg. 1).
 * x (device, in/out): with init = 1 it is overwritten by the uniform start
 * 1/sqrt(N); with init = 0 it holds the caller's start (normalised first,
 * must not be zero); init = 2 is init = 0 plus the warm-start check: the run
 * stops after its second application if that residual is above the first
 * (flags bit 2 set, status OK; the caller restarts from uniform). On return
 * x holds the last unit iterate.
 * tol > 0: stop at the first k with ||x_k - x_{k-1}|| < tol, or after
 * max_iters applications; tol <= 0: exactly max_iters applications (Alg. 1's
 * fixed count). A fixed-count run forms the inner product with the previous
 * iterate (the residual and the Rayleigh quotient) on its first two
 * applications and its last only, the ones it reports: the others do not
 * read the previous iterate. The iterates are the same either way.
 * The iteration runs on the device without host round trips; the call
 * synchronises `stream` once at the end and fills *out (host). out may be
 * NULL: the call then returns as soon as the chain is enqueued (tolerance
 * runs of more than 32 steps still wait on the stream for their stop checks),
 * and no status is read back. */
int stpi_iterate(const stpi_problem *p, const void *f, void *x, int init, int max_iters, double tol,
                 void *ws, size_t ws_bytes, stpi_result *out, void *stream);
/* On a matrix-core variant (stpi_variant_info PIPE 3) a chain of one or more
 * steps runs in product form: the buffers hold w = f .* x * 2^-2e (e from
 * max |f| < 2^e), so each step stages one volume instead of two, and the
 * iterate is w / (f 2^-2e), 0 where f = 0 (which A x is anyway). The final
 * pass forms x from it. Results agree with the plain form to float rounding;
 * after a failed first step (zero or non-finite status) x holds the start
 * masked by f != 0. STPI_NO_PRODUCT=1 in the environment selects the plain
 * form. */

/* ---- the paper's learning objective (SFSeg++), single-field operator --------
 * Float or double device volumes; device scalars are doubles; ws is device
 * scratch of the stated size (STPI_AUX_WS_BYTES always suffices for
 * C <= STPI_MAX_CHANNELS and T <= 1300 frames).
 * stpi_combine_sigmoid_fwd: Eq. 9, f = sigmoid(sum_c w_c fc_c + b), fc
 *   [C][n], w [C], b one value (the standard logistic; the paper prints
 *   exp(+x), a sign slip).
 * stpi_combine_sigmoid_bwd: g_wb[0..C-1] = dL/dw, g_wb[C] = dL/db from dL/df
 *   and the forward's f.
 * stpi_softbin_fwd: Alg. 1, step 3 with the sigmoid's parameter explicit:
 *   b = sigmoid(kappa (sqrt(n) z / ||z|| - theta)), *bnorm = ||b||.
 * stpi_softbin_bwd: given g w.r.t. b / ||b|| (unit = 1, *d = <b / ||b||, g>)
 *   or w.r.t. b (unit = 0), g_y = dL/dy for y = z_prev / ||z_prev|| (the
 *   iterate b was made from) and *d_prev = <y, g_y>, the two inputs of the
 *   adjoint step of the iteration before it.
 * stpi_focal_dice: Eq. 12 per frame with the soft Dice (reading of its
 *   intersection over union): J = sum_t (1 - D_t)^gamma, D_t = (2 sum x gt +
 *   eps) / (sum x + sum gt + eps) over frame t; *loss = J, g_x = dJ/dx.
 *   x [T][plane], gt [T][plane] bytes (0 / nonzero). */
int stpi_combine_sigmoid_fwd(int C, int64_t n, int dtype, const void *fc, const double *w, const double *b, void *f,
                             void *stream);
int stpi_combine_sigmoid_bwd(int C, int64_t n, int dtype, const void *fc, const void *f, const void *g_f,
                             double *g_wb, void *ws, size_t ws_bytes, void *stream);
int stpi_softbin_fwd(int64_t n, int dtype, const void *z, const double *znorm, double kappa, double theta, void *b,
                     double *bnorm, void *ws, size_t ws_bytes, void *stream);
int stpi_softbin_bwd(int64_t n, int dtype, int unit, const void *g, const double *d, const void *b,
                     const double *bnorm, const void *z_prev, const double *znorm_prev, double kappa, void *g_y,
                     double *d_prev, void *ws, size_t ws_bytes, void *stream);
size_t stpi_focal_dice_workspace_bytes(int T);
int stpi_focal_dice(int T, int64_t plane, int dtype, const void *x, const uint8_t *gt, double gamma, double eps,
                    double *loss, void *g_x, void *ws, size_t ws_bytes, void *stream);

/* ---- exact exponential affinity (comparison operator) ----------------------
 * Sec. 3, Eq. 1 before the Taylor approximation, for the exact-vs-approximate
 * comparison of Sec. 4 ("Quantitative analysis"):
 *   z_i = s_i sum_{j in N(i)} s_j exp(-alpha (f_i - f_j)^2) G_ij x_j,
 * alpha >= 0. Not separable: a direct LDS-tiled gather of the whole box per
 * output (meant for small volumes). float or double; r_s <= 8, r_t <= 4
 * (STPI_EUNSUPPORTED otherwise). Arguments and results as the stpi_sfseg_*
 * calls. */
size_t stpi_exp_workspace_bytes(const stpi_problem *p);
int stpi_exp_step(const stpi_problem *p, const void *s, const void *f, double alpha, const void *x, double x_scale,
                  void *z, double *d_sums, void *ws, size_t ws_bytes, void *stream);
int stpi_exp_iterate(const stpi_problem *p, const void *s, const void *f, double alpha, void *x, int init,
                     int max_iters, double tol, void *ws, size_t ws_bytes, stpi_result *out, void *stream);

/* ---- online / partial iteration over sub-windows ---------------------------
 * Sec. 4, "Online vs Offline processing": a long or streaming video is
 * processed in q-frame sub-windows; each window runs a few iterations,
 * starting from the previous window's final solution on the frames the two
 * share. stpi_window_start writes that start vector for a window of
 * pw->T = q frames that lies `shift` frames after the previous one (x_prev,
 * its final unit solution, q frames): frames [0, q - shift) take x_prev's
 * frames [shift, q), the `shift` new frames the uniform start value
 * 1/sqrt(q H W). shift = q (no overlap; x_prev may be NULL) gives the uniform
 * start. Pass x0 to stpi_iterate with init = 0 (it normalises first). The
 * Python driver online.online_iterate runs a whole video this way. */
int stpi_window_start(const stpi_problem *pw, const void *x_prev, int shift, void *x0, void *stream);

/* ---- full SFSeg operator (alpha > 0) ----------------------------------------
 * The paper's update with the first-order Taylor affinity (Sec. 3: Eq. 2,
 * Eq. 5-7; multi-channel form Eq. 10 with s = S_m^p, f = F_m):
 *
 *   z = s (1/alpha - f^2) G*(s x) - s G*(f^2 s x) + 2 s f G*(f s x),
 *   z_i = s_i sum_j s_j [1/alpha - (f_i - f_j)^2] G_ij x_j  = (M x)_i / alpha,
 *
 * with M_ij = s_i s_j [1 - alpha (f_i - f_j)^2] G_ij (Eq. 2), s the unary map
 * raised to the power p (stpi_sfseg_unary) and f the pairwise feature, G as
 * for stpi_iterate. The three filtered fields go through one fused stencil
 * pass. float (STPI_F32) and double (STPI_F64) storage; r_s <= 16, r_t <= 5
 * (STPI_EUNSUPPORTED otherwise). M is symmetric; it is nonnegative (Perron
 * semantics) when s >= 0 and alpha (max f - min f)^2 <= 1, e.g. f in [0, 1]
 * and alpha <= 1; stpi_sfseg_iterate checks this on the device and fails with
 * STPI_EINVAL (flags bit 4) when it does not hold. */

/* s = S^p elementwise (S >= 0, p >= 0; device volumes of n elements). */
int stpi_sfseg_unary(int64_t n, int dtype, const void *S, double p, void *s, void *stream);
/* Device workspace of stpi_sfseg_step / stpi_sfseg_iterate (0 if p is invalid
 * or unsupported). */
size_t stpi_sfseg_workspace_bytes(const stpi_problem *p);
/* One application, unnormalised: z as above with x scaled by x_scale;
 * d_sums[0] = sum z^2, d_sums[1] = sum z .* x * x_scale (device doubles).
 * z must not alias s, f or x. */
int stpi_sfseg_step(const stpi_problem *p, const void *s, const void *f, double alpha, const void *x,
                    double x_scale, void *z, double *d_sums, void *ws, size_t ws_bytes, void *stream);
/* Power iteration with the full operator (Eq. 7 then Eq. 8; Alg. 1 without
 * its soft-binarisation): x in/out, init = 1 uniform start, init = 0 the
 * caller's x (Alg. 1 starts from the unary map: pass it as x). Stopping, the
 * result and the residual as stpi_iterate. Synchronises `stream`. */
int stpi_sfseg_iterate(const stpi_problem *p, const void *s, const void *f, double alpha, void *x, int init,
                       int max_iters, double tol, void *ws, size_t ws_bytes, stpi_result *out, void *stream);

/* ---- kernel variants ------------------------------------------------------
 * Each storage type has a list of compiled step kernels (radii RS >= r_s,
 * RT >= r_t, tile TH x TW, NTHR threads, RY rows per y-pass item, QX outputs
 * per x-pass item). By default
 * the library picks the cheapest eligible one (or the autotuned one). */

/* Number of compiled variants for dtype (0 for an unknown dtype). */
int stpi_variant_count(int dtype);
/* info[0..8] = RS, RT, TH, TW, NTHR, RY, QX, OCC (min waves per SIMD), PIPE of
 * variant `index` (tile loop: 0 plain, 1 software-pipelined, 2 straight-line,
 * 3 matrix-core spatial passes); STPI_EINVAL if out of range. */
int stpi_variant_info(int dtype, int index, int32_t info[9]);
/* Launch shape the step of problem p uses with variant `variant` (-1: the
 * variant stpi_step would choose): info[0] = variant index, info[1] = tiles
 * per frame, info[2] = frame segments per tile (a tile's frames are split
 * when the chip holds more resident workgroups than there are tiles, and a
 * short clip's frames when that shortens the slowest segment by two frame
 * steps or more; each segment re-reads r_t frames on each inner side, and
 * a last segment that starts after frame 0 is walked backward in time, which
 * changes only the order of its sums), info[3] = workgroups per
 * CU that fit at once, info[4] = workgroups launched. Queries the current
 * device. STPI_EINVAL / STPI_EUNSUPPORTED as for stpi_step. */
int stpi_launch_shape(const stpi_problem *p, int variant, int32_t info[5]);
/* Force variant `index` for every later call in the process (-1: automatic
 * choice). A forced variant whose radii are too small makes calls fail with
 * STPI_EUNSUPPORTED. Not thread-safe against concurrent launches. */
int stpi_set_variant(int index);

/* Average duration in milliseconds of the step kernel alone (no reduction
 * epilogue launch), measured with HIP events recorded on `stream` around
 * `reps` back-to-back launches of variant `variant` (-1: the variant
 * stpi_step would use) in single-step mode z = A x. f, x, z are device volumes
 * as for stpi_step; ws as for stpi_step. Synchronises `stream`. Used by the
 * benchmark and the autotuner. */
int stpi_time_step(const stpi_problem *p, const void *f, const void *x, void *z, void *ws, size_t ws_bytes,
                   int variant, int reps, void *stream, double *avg_ms);

/* Average duration in milliseconds of one step of an iteration chain, as
 * stpi_iterate runs it (the step kernel with its fused finalisation; on a
 * matrix-core variant the product form, see stpi_iterate), measured with HIP
 * events on `stream` around `reps` back-to-back steps of a fixed-count chain
 * from the uniform start (steps 2 .. reps + 1 of a chain of reps + 2, so all
 * but the first timed step skip the previous iterate as stpi_iterate's
 * fixed-count runs do). f: device volume of p->dtype; x: a device volume of
 * p->dtype used as scratch (overwritten); ws as for stpi_iterate. variant: as
 * for stpi_time_step. *product_form (if not NULL) receives 1 when the product
 * form ran. Synchronises `stream`. Used by the benchmark. */
int stpi_time_chain_step(const stpi_problem *p, const void *f, void *x, void *ws, size_t ws_bytes, int variant,
                         int reps, void *stream, double *avg_ms, int *product_form);

/* ---- batched clips --------------------------------------------------------
 * Many clips of different length and frame size iterated together, all with
 * the same filter. Their volumes sit in flat device buffers at per-clip
 * element offsets (non-overlapping; 256-byte aligned offsets are best). Each
 * iteration is one persistent launch whose workgroups pull tiles from a work
 * list (longest clips first); every clip keeps its own state, stops on its own
 * (tolerance or cap) and is skipped afterwards. The whole chain of max_iters
 * iterations is captured once per (buffers, stream) as a HIP graph and
 * replayed with a single graph launch. */

typedef struct stpi_clip {
    int64_t offset;  /* element offset of the clip in the flat buffers */
    int32_t T, H, W;
    int32_t reserved;
} stpi_clip;

typedef struct stpi_plan stpi_plan;

/* Builds a plan: validates the clips, picks the step kernel variant (the
 * autotuned one for the frame size carrying the most voxels, else the
 * cheapest eligible one), orders the tile list and uploads the clip and tile
 * tables (the only device allocations, made here, not on the hot path).
 * *out receives the plan (owned by the caller, free with stpi_plan_destroy). */
int stpi_batch_plan(const stpi_clip *clips, int nclips, float sigma_s, float sigma_t, int r_s, int r_t, int dtype,
                    stpi_plan **out);
/* Device workspace stpi_batch_iterate needs (0 for NULL). */
size_t stpi_batch_workspace_bytes(const stpi_plan *plan);
/* info[0..10] = nclips, ntiles, persistent grid size, RS, RT, TH, TW, NTHR, RY, QX,
 * PIPE (0: plain tile loop, 1: software-pipelined, 3: matrix-core, whose chains
 * run in product form as stpi_iterate describes, per clip). */
int stpi_batch_info(const stpi_plan *plan, int32_t info[11]);
/* Power iteration of every clip (as stpi_iterate, per clip): x_flat is in/out,
 * init = 1 overwrites each clip with the uniform start, init = 0 uses x_flat.
 * init = 2 is init = 0 with the warm-start rule applied per clip on the
 * device: a clip whose residual after the second application exceeds the
 * first restarts from the uniform start (flags bit 2 set; its iteration count
 * includes the two discarded applications; max_iters bounds the total).
 * Stops each clip at its first residual < tol (tol > 0) or after max_iters;
 * a clip that stopped costs the following steps nothing (every step claims
 * tiles from the list of clips still iterating).
 * per_clip: host array of nclips results. Synchronises `stream` once. Calls
 * with a NULL stream run without graph capture. */
int stpi_batch_iterate(stpi_plan *plan, const void *f_flat, void *x_flat, int init, int max_iters, double tol,
                       void *ws, size_t ws_bytes, stpi_result *per_clip, void *stream);
void stpi_plan_destroy(stpi_plan *plan);

/* ---- autotuner -------------------------------------------------------------
 * stpi_autotune times every compiled variant eligible for `p` as a step of an
 * iteration chain (stpi_time_chain_step, reps steps each, on temporary device
 * buffers it allocates and frees),
 * records the fastest for (device arch, dtype, r_s, r_t, H, W), and writes the
 * whole table to cache_path (if not NULL). Later calls for that key use the
 * recorded variant. Synchronises the device. */
int stpi_autotune(const stpi_problem *p, const char *cache_path, int reps, int32_t *best_variant, double *best_ms);
/* Merges a table written by stpi_autotune into the process's table. */
int stpi_autotune_load(const char *path);
/* Forgets every recorded choice. */
void stpi_autotune_clear(void);

/* ---- differentiation path ---------------------------------------------------
 * The gradient of a loss through the whole normalised iteration ("propagating
 * the gradient of the loss through the full spectral algorithm", Sec. 1 and
 * Sec. 3.4), so that per-channel combination weights can be learned end to
 * end. Iterates live on a tape unnormalised: x_k = z_k / norm_k, with norm_k
 * a device double. All scalars (norms, inner products, loss) stay in device
 * memory so the whole forward and backward run without host round trips.
 * Storage types with adjoint kernels: STPI_F32, STPI_F64. */

#define STPI_MAX_CHANNELS 64
/* Device workspace the auxiliary reductions (dot, combine_bwd, bce) need. */
#define STPI_AUX_WS_BYTES (512 * 1024)

/* x0 <- 1 (every voxel), *norm0 <- sqrt(T H W): the uniform unit start
 * 1/sqrt(N) on the tape (Sec. 4, uniform initialisation). */
int stpi_train_init(const stpi_problem *p, void *x0, double *norm0, void *stream);

/* One tape step (Eq. 4 + Eq. 8 without the division):
 *   x = z_in / *norm_in, z_out = f .* G * (f .* x), v_out = G * (f .* x)
 *   (v_out may be NULL), *norm_out = ||z_out||.
 * z_out and v_out must not alias the inputs. ws: stpi_workspace_bytes(p). */
int stpi_train_step(const stpi_problem *p, const void *f, const void *z_in, const double *norm_in, void *z_out,
                    void *v_out, double *norm_out, void *ws, size_t ws_bytes, void *stream);

/* Adjoint of tape step k. Inputs: f; z_k, *norm_k (x_k = z_k / norm_k);
 * z_k1, *norm_k1 (x_{k+1}); v_k = G (f .* x_k) saved by the forward step;
 * g_k1 = dL/dx_{k+1}; *d_k1 = <x_{k+1}, g_k1>. Outputs:
 *   g_k = f .* G (f .* g_z),  g_z = (g_k1 - x_{k+1} d_k1) / norm_k1,
 *   g_f += v_k .* g_z + x_k .* G (f .* g_z)     (accumulated in place),
 *   *d_k = <x_k, g_k>  (the d of step k - 1).
 * g_k must not alias another argument. ws: stpi_workspace_bytes(p). */
int stpi_adjoint_step(const stpi_problem *p, const void *f, const void *z_k, const double *norm_k, const void *z_k1,
                      const double *norm_k1, const void *v_k, const void *g_k1, const double *d_k1, void *g_k,
                      void *g_f, double *d_k, void *ws, size_t ws_bytes, void *stream);

/* x = z / *norm over n elements (x may alias z). */
int stpi_normalize(int64_t n, int dtype, const void *z, const double *norm, void *x, void *stream);

/* *out = <a, b> / (a_norm ? *a_norm : 1) over n elements (double sums of exact
 * double products). ws: STPI_AUX_WS_BYTES. */
int stpi_dot(int64_t n, int dtype, const void *a, const double *a_norm, const void *b, double *out, void *ws,
             size_t ws_bytes, void *stream);

/* Multi-channel combination (the learnable channel weighting of Eq. 9, in the
 * convex form f = sum_c softmax(w)_c fc_c): fc is [C][n], w holds C double
 * logits in device memory, f is [n]. 1 <= C <= STPI_MAX_CHANNELS. */
int stpi_combine_fwd(int C, int64_t n, int dtype, const void *fc, const double *w, void *f, void *stream);

/* g_w[c] (device doubles) = dL/dw_c given g_f = dL/df:
 * g_a_c = <g_f, fc_c>, g_w = softmax(w) .* (g_a - <softmax(w), g_a>).
 * ws: STPI_AUX_WS_BYTES. */
int stpi_combine_bwd(int C, int64_t n, int dtype, const void *fc, const double *w, const void *g_f, double *g_w,
                     void *ws, size_t ws_bytes, void *stream);

/* Binary cross-entropy of the soft segmentation against a ground-truth mask:
 * y = clip(x / max(x), 1e-7, 1 - 1e-7), *loss = mean(-(gt log y + (1 - gt) log(1 - y))),
 * g_x = dL/dx (clipped entries pass no gradient; the max-normalisation term goes
 * to the first maximal element). gt: n bytes, 0 or nonzero. ws: STPI_AUX_WS_BYTES. */
int stpi_bce(int64_t n, int dtype, const void *x, const uint8_t *gt, double *loss, void *g_x, void *ws,
             size_t ws_bytes, void *stream);

/* AdamW (Eq. 13, decoupled weight decay, with AMSGrad when amsgrad != 0) on n
 * parameters of dtype STPI_F32 or STPI_F64 in device memory (w, g, m, v, vmax
 * all of that type), step >= 1 (1-based, for the bias corrections):
 * w <- w (1 - lr wd); m <- b1 m + (1 - b1) g; v <- b2 v + (1 - b2) g^2;
 * vmax <- max(vmax, v); w <- w - lr (m / (1 - b1^step)) / (sqrt(vmax / (1 - b2^step)) + eps).
 * vmax may be NULL when amsgrad == 0. */
int stpi_adamw(int64_t n, int dtype, void *w, const void *g, void *m, void *v, void *vmax, int step, double lr,
               double beta1, double beta2, double eps, double weight_decay, int amsgrad, void *stream);

/* ---- two-level start: grid transfer -------------------------------------------
 * The slowest modes of the power iteration on multi-object clips compete
 * between objects far apart; an iteration on a coarse grid (cheap: sy^2 st
 * times fewer voxels) resolves them, and its eigenvector, carried back to the
 * full grid, starts the full iteration. Not part of the paper; its own warm
 * start reuses the previous sub-window's solution (Sec. 4, "Online vs Offline processing").
 * Coarse size: Tc = ceil(T / st), Hc = ceil(H / sy), Wc = ceil(W / sy). */
/* out[tc][yc][xc] = mean of in[t][y][x] over the voxels of block
 * [tc st, (tc+1) st) x [yc sy, (yc+1) sy) x [xc sy, (xc+1) sy) inside the
 * volume (partial blocks at the far edges average what exists). in: T x H x W,
 * out: Tc x Hc x Wc, both of storage type dtype, device, out must not alias in.
 * Asynchronous on `stream`. STPI_EINVAL for bad sizes, factors < 1, NULL or
 * aliased buffers (checked before launch). */
int stpi_downsample(int T, int H, int W, int sy, int st, int dtype, const void *in, void *out, void *stream);
/* out (T x H x W) = up(in) (Tc x Hc x Wc), times mul[i] if mul is not NULL.
 * mode 0: the coarse cell holding the voxel; mode 1: cell-centred trilinear,
 * coarse coordinate c = (i + 1/2) / s - 1/2 per axis, clamped to [0, n - 1].
 * out must not alias in or mul. Asynchronous; errors as stpi_downsample. */
int stpi_upsample(int T, int H, int W, int sy, int st, int mode, int dtype, const void *in, const void *mul, void *out,
                  void *stream);
/* The coarse problem of the two-level start (host only, no device work):
 * coarse size as above, the kernel's sigmas divided by the factors
 * (sigma_s / sy, sigma_t / st) and its radii rounded up (ceil(r_s / sy),
 * ceil(r_t / st)), the dtype kept. STPI_EINVAL for NULL pointers, sizes or
 * factors < 1, sigmas <= 0 or negative radii. */
int stpi_coarse_problem(const stpi_problem *fine, int sy, int st, stpi_problem *coarse);
/* y[i] = x[i] * s, times *s_dev as well when s_dev (a device double) is not
 * NULL; formed in double and rounded to the storage type once. n elements of
 * storage type dtype, device buffers; y may be x. Used for the start's O(1)
 * scaling for the net and for a loss gradient times the incoming gradient.
 * Asynchronous on `stream`; STPI_EINVAL for n < 0, an unknown dtype or NULL
 * buffers (n > 0). */
int stpi_scale(int64_t n, int dtype, const void *x, double s, const double *s_dev, void *y, void *stream);

/* ---- learned warm start ------------------------------------------------------
 * A small 3D convolutional network predicts the start vector of the iteration
 * from f (the paper's own warm start is the previous sub-window's solution,
 * Sec. 4, "Online vs Offline processing"; here a network trained on eigenvectors of the plain method plays
 * that role). Four 'same' 3x3x3 convolutions with zero padding and bias,
 * 1 -> 16 -> 16 -> 16 -> 1 channels, ReLU between layers; bfloat16 weights and
 * activations, FP32 accumulation; the 16 -> 16 layers run on the matrix cores.
 * Parameters are FP32 masters (stpi_net_param_count() floats, PyTorch conv3d
 * order [Cout][Cin][3][3][3] per layer: w1 b1 w2 b2 w3 b3 w4 b4); kernels read
 * a prepared bfloat16 copy (stpi_net_prep_bytes() bytes) made by
 * stpi_net_prepare. f and y are FP32 [T][H][W] volumes; ws holds the
 * activations kept for the backward pass (stpi_net_workspace_bytes). */
int stpi_net_param_count(void);
size_t stpi_net_prep_bytes(void);
size_t stpi_net_workspace_bytes(const stpi_problem *p);
/* prep <- bfloat16 operand layouts of master (device). */
int stpi_net_prepare(const float *master, void *prep, void *stream);
/* y = net(f); the activations stay in ws for stpi_net_backward. */
int stpi_net_forward(const stpi_problem *p, const float *f, const void *prep, float *y, void *ws, size_t ws_bytes,
                     void *stream);
/* After stpi_net_forward with the same ws: *loss = mean((y - x_star sqrt(N))^2)
 * (x_star: the target unit eigenvector) and grad (same layout as the masters,
 * overwritten) = dloss/dparameters. */
int stpi_net_backward(const stpi_problem *p, const float *f, const void *prep, const float *y, const float *x_star,
                      double *loss, float *grad, void *ws, size_t ws_bytes, void *stream);
/* x0 = max(y, 0) + eps (the iteration normalises its start vector). */
int stpi_net_warm_start(int64_t n, const float *y, float eps, float *x0, void *stream);

#ifdef __cplusplus
}
#endif

#endif /* STPI_H */
