// Per-storage-type entry points of the kernel set (one translation unit per type).
#pragma once

#include "adjoint.hpp"
#include "batch.hpp"
#include "forward.hpp"

namespace stpi {

struct DtypeOps {
    size_t elem;                 // bytes per stored element
    const Variant *variants;     // compiled step kernels
    int nvariants;
    hipError_t (*fill_ones)(void *x, size_t n, hipStream_t);
    hipError_t (*sumsq)(const void *x, size_t n, double *partials, hipStream_t);
    hipError_t (*normalize)(void *x, const void *buf1, size_t n, const DevState *s, hipStream_t);
    // *out = max(*out, max |f| or max |f x|) as float bits (matrix-core step variants)
    hipError_t (*bound)(size_t n, const void *f, const void *x, uint32_t *out, hipStream_t);
    // product-form chains: start (w = f x g into buf1) and final pass (x = unit iterate)
    hipError_t (*to_product)(const void *f, const void *x, void *buf1, size_t n, DevState *s, hipStream_t);
    hipError_t (*from_product)(void *x, const void *buf1, const void *f, size_t n, const DevState *s, hipStream_t);
    // differentiation path (null where a storage type does not provide it)
    const AdjVariant *adj_variants;
    int nadj;
    hipError_t (*combine_fwd)(int C, size_t n, const void *fc, const double *w, void *f, hipStream_t);
    hipError_t (*combine_bwd)(int C, size_t n, const void *fc, const void *gf, double *partials, hipStream_t);
    hipError_t (*scale_by_norm)(size_t n, const void *z, const double *norm, void *x, hipStream_t);
    hipError_t (*dot)(size_t n, const void *a, const void *b, double *partials, hipStream_t);
    hipError_t (*train_init)(size_t n, void *x, double *norm, hipStream_t);
    hipError_t (*maxarg)(size_t n, const void *x, double *partials, hipStream_t);
    hipError_t (*bce)(size_t n, const void *x, const uint8_t *gt, const double *scalars, void *gx, double *partials,
                      hipStream_t);
    hipError_t (*bce_finalize)(size_t n, int nblocks, const double *partials, const double *scalars, void *gx,
                               double *loss, hipStream_t);
    // batched chain
    const BatchVariant *batch_variants;
    int nbatch;
    hipError_t (*batch_fill)(void *x, const ClipDesc *clips, int nclips, hipStream_t);
    hipError_t (*batch_sumsq)(const void *x, const ClipDesc *clips, int nclips, double *partials, hipStream_t);
    hipError_t (*batch_normalize)(void *x, const void *buf1, const ClipDesc *clips, const DevState *states,
                                  int nclips, hipStream_t);
    // matrix-core batch variants (product form): per-clip bound, start and final pass
    hipError_t (*batch_bound)(const void *f, const ClipDesc *clips, DevState *states, int nclips, hipStream_t);
    hipError_t (*batch_to_product)(const void *f, const void *x, void *buf1, const ClipDesc *clips, DevState *states,
                                   int nclips, hipStream_t);
    hipError_t (*batch_from_product)(void *x, const void *buf1, const void *f, const ClipDesc *clips,
                                     const DevState *states, int nclips, hipStream_t);
    // plain-form batch: uniform restart of the clips whose warm start was rejected
    hipError_t (*batch_refill)(void *x, void *buf1, const ClipDesc *clips, const DevState *states, int nclips,
                               hipStream_t);
};

const DtypeOps *dtype_ops_f32();
const DtypeOps *dtype_ops_bf16();
const DtypeOps *dtype_ops_f64();

}  // namespace stpi
