// Non-template kernels of the batched chain and their host-side launchers.
#include "batch.hpp"
#include "host_internal.hpp"

namespace stpi {

// Per-clip start: uniform (scale 1/sqrt(N_clip)) or the caller's vector
// (scale from the per-clip sum of squares, computed afterwards).
__global__ void batch_init_kernel(DevState *states, const ClipDesc *clips, int nclips, double tol, int max_iters,
                                  int uniform, int check_rise, int pform, BatchCtl *ctl) {
    const int c = blockIdx.x * blockDim.x + threadIdx.x;
    if (c == 0) {
        ctl->next_tile = 0u;
        ctl->done_clips = max_iters <= 0 ? (uint32_t)nclips : 0u;
    }
    if (c >= nclips) return;
    const ClipDesc cd = clips[c];
    DevState *s = states + c;
    s->scale = uniform ? 1.0 / sqrt((double)cd.T * cd.H * cd.W) : 1.0;
    s->residual = 0.0;
    s->lambda = 0.0;
    s->rayleigh = 0.0;
    s->tol = tol;
    s->iters = 0;
    s->done = max_iters <= 0 ? 1 : 0;
    s->cur = 0;
    s->flags = 0u;
    s->max_iters = max_iters;
    s->converged = 0;
    s->arrive = 0u;
    s->ubound = 0u;
    s->wmax[0] = s->wmax[1] = 0u;
    s->refill = 0;
    s->first_res[0] = s->first_res[1] = 0.0;
    s->check_rise = check_rise;
    s->pform = uniform && pform ? 2 : 0;
}

__global__ void batch_state_from_norm_kernel(const double *partials, DevState *states, BatchCtl *ctl) {
    __shared__ double red[CHAIN_THREADS / 64];
    const int c = blockIdx.x;
    double a = 0.0;
    for (int i = threadIdx.x; i < BATCH_NORM_BLOCKS; i += CHAIN_THREADS)
        a += partials[2 * ((size_t)c * BATCH_NORM_BLOCKS + i)];
    const double ss = block_sum<CHAIN_THREADS>(a, red);
    if (threadIdx.x == 0) {
        DevState *s = states + c;
        const double nrm = sqrt(ss);
        if (s->done) return;
        if (!isfinite(nrm) || nrm == 0.0) {
            s->flags |= isfinite(nrm) ? FLAG_ZERO : FLAG_NONFINITE;
            s->done = 1;
            atomicAdd(&ctl->done_clips, 1u);
        } else {
            s->scale = 1.0 / nrm;
        }
    }
}

__global__ void batch_finalize_kernel(const double *partials, const ClipDesc *clips, DevState *states,
                                      BatchCtl *ctl) {
    __shared__ double red[CHAIN_THREADS / 64];
    const int c = blockIdx.x;
    if (c == 0 && threadIdx.x == 0) ctl->next_tile = 0u;  // the step that wrote partials has finished
    DevState *s = states + c;
    if (s->done) return;
    const ClipDesc cd = clips[c];
    double a = 0.0, b = 0.0;
    for (int t = cd.tile_begin + threadIdx.x; t < cd.tile_end; t += CHAIN_THREADS) {
        a += partials[2 * (size_t)t];
        b += partials[2 * (size_t)t + 1];
    }
    const double p1 = block_sum<CHAIN_THREADS>(a, red);
    const double p2 = block_sum<CHAIN_THREADS>(b, red);
    if (threadIdx.x == 0) finalize_state(s, p1, p2, ctl, (double)cd.T * cd.H * cd.W);
}

// Rebuilds the list of clips still iterating (in tile-list order, clip_order)
// and the exclusive prefix sums of their tile counts, which the next step's
// workgroups claim tiles from: clips that stopped cost the step nothing.
// One workgroup of COMPACT_THREADS.
constexpr int COMPACT_THREADS = 256;
__global__ void batch_compact_kernel(const DevState *states, const ClipDesc *clips, const int32_t *clip_order,
                                     int nclips, int32_t *active_clip, int32_t *active_cum, BatchCtl *ctl) {
    __shared__ long long scan[COMPACT_THREADS];
    __shared__ long long base;
    const int tid = threadIdx.x;
    if (tid == 0) base = 0;
    __syncthreads();
    for (int c0 = 0; c0 < nclips; c0 += COMPACT_THREADS) {
        const int i = c0 + tid;
        int c = -1;
        long long v = 0;  // (tile count << 20) | 1 for an active clip
        if (i < nclips) {
            c = clip_order[i];
            if (!states[c].done) v = ((long long)(clips[c].tile_end - clips[c].tile_begin) << 20) | 1;
        }
        scan[tid] = v;
        __syncthreads();
        for (int off = 1; off < COMPACT_THREADS; off <<= 1) {
            const long long add = tid >= off ? scan[tid - off] : 0;
            __syncthreads();
            scan[tid] += add;
            __syncthreads();
        }
        const long long ex = base + scan[tid] - v;  // exclusive prefix, both fields
        if (v) {
            const int slot = (int)(ex & ((1 << 20) - 1));
            active_clip[slot] = c;
            active_cum[slot] = (int32_t)(ex >> 20);
        }
        __syncthreads();
        if (tid == COMPACT_THREADS - 1) base += scan[tid];
        __syncthreads();
    }
    if (tid == 0) {
        ctl->n_active = (uint32_t)(base >> 20);
        ctl->n_clips_active = (uint32_t)(base & ((1 << 20) - 1));
    }
}

hipError_t launch_batch_init(DevState *states, const ClipDesc *clips, int nclips, double tol, int max_iters,
                             int uniform, int check_rise, int pform, BatchCtl *ctl, hipStream_t st) {
    hipLaunchKernelGGL(batch_init_kernel, dim3((nclips + 63) / 64), dim3(64), 0, st, states, clips, nclips, tol,
                       max_iters, uniform, check_rise, pform, ctl);
    return hipGetLastError();
}

hipError_t launch_batch_compact(const DevState *states, const ClipDesc *clips, const int32_t *clip_order, int nclips,
                                int32_t *active_clip, int32_t *active_cum, BatchCtl *ctl, hipStream_t st) {
    hipLaunchKernelGGL(batch_compact_kernel, dim3(1), dim3(COMPACT_THREADS), 0, st, states, clips, clip_order, nclips,
                       active_clip, active_cum, ctl);
    return hipGetLastError();
}

hipError_t launch_batch_state_from_norm(const double *partials, DevState *states, int nclips, BatchCtl *ctl,
                                        hipStream_t st) {
    hipLaunchKernelGGL(batch_state_from_norm_kernel, dim3(nclips), dim3(CHAIN_THREADS), 0, st, partials, states,
                       ctl);
    return hipGetLastError();
}

hipError_t launch_batch_finalize(const double *partials, const ClipDesc *clips, DevState *states, int nclips,
                                 BatchCtl *ctl, hipStream_t st) {
    hipLaunchKernelGGL(batch_finalize_kernel, dim3(nclips), dim3(CHAIN_THREADS), 0, st, partials, clips, states,
                       ctl);
    return hipGetLastError();
}

}  // namespace stpi
