// Shared device-side types for the stpi kernels (gfx950).
#pragma once

#include <hip/hip_runtime.h>
#include <stddef.h>
#include <stdint.h>

namespace stpi {

// bfloat16 storage: the upper 16 bits of an IEEE binary32 value.
struct bf16 {
    uint16_t bits;
};

__device__ __forceinline__ float ld(const float *p) { return *p; }
__device__ __forceinline__ double ld(const double *p) { return *p; }
__device__ __forceinline__ float ld(const bf16 *p) {
    return __uint_as_float(((uint32_t)p->bits) << 16);
}

// Round-to-nearest-even float -> bfloat16 (NaN stays NaN): the hardware
// conversion, one instruction per pair.
__device__ __forceinline__ uint16_t f32_to_bf16_bits(float v) { return __builtin_bit_cast(uint16_t, (__bf16)v); }
__device__ __forceinline__ uint32_t f32x2_to_bf16x2_bits(float a, float b) {
    typedef float f2_t __attribute__((ext_vector_type(2)));
    typedef __bf16 b2_t __attribute__((ext_vector_type(2)));
    const f2_t v = {a, b};
    return __builtin_bit_cast(uint32_t, __builtin_convertvector(v, b2_t));
}

__device__ __forceinline__ void st(float *p, float v) { *p = v; }
__device__ __forceinline__ void st(double *p, double v) { *p = v; }
__device__ __forceinline__ void st(bf16 *p, float v) { p->bits = f32_to_bf16_bits(v); }

// The value a store of v would leave in memory, read back in compute precision.
__device__ __forceinline__ float stored_value(const float *, float v) { return v; }
__device__ __forceinline__ double stored_value(const double *, double v) { return v; }
__device__ __forceinline__ float stored_value(const bf16 *, float v) {
    return __uint_as_float(((uint32_t)f32_to_bf16_bits(v)) << 16);
}

// Compute type for a storage type.
template <class ST> struct Compute { using type = float; };
template <> struct Compute<double> { using type = double; };

// Iteration state kept in device memory so that a whole iteration chain runs
// without host round trips. The stored iterate is unnormalised; the unit
// iterate is scale * stored.
struct DevState {
    double scale;      // 1 / ||stored iterate||
    double residual;   // ||x_k - x_{k-1}|| of the last step
    double lambda;     // ||A x_{k-1}||
    double rayleigh;   // <x_{k-1}, A x_{k-1}>
    double tol;        // <= 0: run a fixed number of steps
    int32_t iters;     // applications of A done
    int32_t done;      // 1: converged or stopped, further steps are no-ops
    int32_t cur;       // 0: iterate lives in buffer 0 (the caller's x), 1: in buffer 1
    uint32_t flags;    // bit 0 zero norm, bit 1 non-finite
    int32_t max_iters;
    int32_t converged;
    uint32_t arrive;   // workgroups of the running step that stored their partial sums
    uint32_t ubound;   // float bits of max |f| (matrix-core step variants)
    double first_res[2];  // residuals after the chain's first and second steps
    int32_t check_rise;   // 1: stop after the second step if its residual is above the first's
    // 0: the buffers hold the iterate itself. Product form (matrix-core chain
    // steps): 1: the current buffer holds w = f x g (see FwdOpP), 2: uniform
    // start, no step taken yet (the iterate is the constant 1, w = f itself).
    int32_t pform;
    // Product form: float bits of max |w| over buffer 0 / buffer 1 (the
    // buffer a step writes collects it; the step's finalisation clears the
    // entry of the buffer it read, which the next step writes).
    uint32_t wmax[2];
    // Batched chains, plain form: 1 after a rejected warm start until the
    // clip's buffer has been refilled with the uniform start.
    int32_t refill;
};

static_assert(sizeof(DevState) <= 256, "the iteration state lives in a 256-byte workspace slot");

constexpr uint32_t FLAG_ZERO = 1u;
constexpr uint32_t FLAG_NONFINITE = 2u;
constexpr uint32_t FLAG_ROSE = 4u;  // the check_rise rule fired (not an error): single clip stops, batched clip restarts

// Exponent e of a bound (bound < 2^e, from frexp), clamped to [-lim, lim];
// 0 for a zero or non-finite bound.
__device__ __forceinline__ int bound_exponent(float bound, int lim) {
    int e = 0;
    if (bound > 0.f && bound <= 3.0e38f) (void)frexpf(bound, &e);
    return e < -lim ? -lim : (e > lim ? lim : e);
}
// Product-form chains keep 2^(+-2e) normal floats.
constexpr int PRODUCT_ELIM = 60;

// An empty partial-sum slot of a step whose last workgroup finalises it: a
// signalling-NaN pattern that arithmetic never produces (its NaNs are quiet).
// Each workgroup overwrites its slot with an agent-scope atomic store; the last
// workgroup reads every slot until it no longer holds this pattern (so it sees
// the stored value by the coherence of that one location, without a cache
// write-back) and puts the pattern back for the next step.
constexpr uint64_t PARTIAL_EMPTY = 0x7ff4dead5a17ab1eull;
// Reads of one slot before the wait is abandoned (never reached in practice:
// the arrival counter is only bumped after the slot's store has completed).
constexpr int PARTIAL_SPIN_LIMIT = 1 << 20;
constexpr uint32_t FLAG_SYNC = 8u;  // a partial sum never arrived (see PARTIAL_SPIN_LIMIT)
constexpr uint32_t FLAG_AFFINITY = 16u;  // full operator: a Taylor affinity could be negative (see sfseg.hip)

// Workgroup size and summation order of the per-step reduction of partial
// sums: thread i < FINAL_THREADS adds entries i, i + FINAL_THREADS, ... in
// turn, then the workgroup tree of block_sum.
constexpr int FINAL_THREADS = 256;

// Step finalisation from the reduced sums P1 = sum z * x_stored and
// P2 = sum z^2: n = ||z||, x_{k+1} = z / n (Eq. 8), cos = <x_{k+1}, x_k> =
// scale * P1 / n, residual = sqrt(2 - 2 cos), and the stopping rules.
__device__ __forceinline__ void step_finalize(DevState *s, double p1, double p2) {
    const double scale = s->scale;
    const double nz = sqrt(p2);
    if (!isfinite(nz) || !isfinite(p1)) {
        s->flags |= FLAG_NONFINITE;
        s->done = 1;
        return;
    }
    if (nz == 0.0) {
        s->flags |= FLAG_ZERO;
        s->done = 1;
        return;
    }
    const double c = scale * p1 / nz;
    s->rayleigh = scale * p1;
    s->lambda = nz;
    s->residual = sqrt(fmax(0.0, 2.0 - 2.0 * c));
    s->scale = 1.0 / nz;
    s->wmax[s->cur] = 0u;  // the buffer just read is the next step's output
    s->cur ^= 1;
    s->iters += 1;
    if (s->pform == 2) s->pform = 1;
    if (s->iters <= 2) s->first_res[s->iters - 1] = s->residual;
    if (s->check_rise && s->iters == 2 && !(s->first_res[1] <= s->first_res[0])) {
        s->flags |= FLAG_ROSE;
        s->done = 1;
        return;
    }
    if (s->tol > 0.0 && s->residual < s->tol) {
        s->converged = 1;
        s->done = 1;
    }
    if (s->iters >= s->max_iters) s->done = 1;
}

// Sum of a double over a workgroup (fixed shuffle/LDS tree: deterministic).
template <int NTHR>
__device__ __forceinline__ double block_sum(double v, double *lds) {
#pragma unroll
    for (int off = 32; off >= 1; off >>= 1) v += __shfl_xor(v, off, 64);
    constexpr int NW = NTHR / 64;
    const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
    __syncthreads();
    if (lane == 0) lds[wid] = v;
    __syncthreads();
    double s = 0.0;
    if (threadIdx.x == 0) {
#pragma unroll
        for (int i = 0; i < NW; ++i) s += lds[i];
    }
    return s;  // valid in thread 0 only
}

// Maximum of a non-negative float over a workgroup (valid in thread 0).
template <int NTHR>
__device__ __forceinline__ float block_max(float v, float *lds) {
#pragma unroll
    for (int off = 32; off >= 1; off >>= 1) v = fmaxf(v, __shfl_xor(v, off, 64));
    constexpr int NW = NTHR / 64;
    const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
    __syncthreads();
    if (lane == 0) lds[wid] = v;
    __syncthreads();
    float m = 0.f;
    if (threadIdx.x == 0) {
#pragma unroll
        for (int i = 0; i < NW; ++i) m = fmaxf(m, lds[i]);
    }
    return m;
}

// Reads partial-sum slot i of a step finalised by its last workgroup (see
// PARTIAL_EMPTY) and empties it again; *late is set if it never arrived.
__device__ __forceinline__ double take_partial(double *slot, bool *late) {
    uint64_t *w = reinterpret_cast<uint64_t *>(slot);
    uint64_t v = __hip_atomic_load(w, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    for (int k = 0; v == PARTIAL_EMPTY && k < PARTIAL_SPIN_LIMIT; ++k) {
        __builtin_amdgcn_s_sleep(1);
        v = __hip_atomic_load(w, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    }
    if (v == PARTIAL_EMPTY) *late = true;
    __hip_atomic_store(w, PARTIAL_EMPTY, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    return __longlong_as_double((long long)v);
}

}  // namespace stpi
