// Instantiates the kernel set for one storage type. Included once per type by
// kernels_<type>.hip with STPI_ST (storage type), STPI_NAME (suffix) and
// STPI_VARIANTS(X) (the compiled (RS, RT, TH, TW, NTHR, RY, QX, OCC, PIPE) list) defined.
#pragma once

#include "aux.hpp"
#include "batch.hpp"
#include "chain.hpp"
#include "dtype_ops.hpp"

namespace stpi {
namespace {

using ST_ = STPI_ST;

hipError_t fill_ones_impl(void *x, size_t n, hipStream_t s) {
    hipLaunchKernelGGL(fill_ones_kernel<ST_>, dim3(1024), dim3(256), 0, s, (ST_ *)x, n);
    return hipGetLastError();
}

hipError_t sumsq_impl(const void *x, size_t n, double *partials, hipStream_t s) {
    hipLaunchKernelGGL(sumsq_kernel<ST_>, dim3(NORM_BLOCKS), dim3(CHAIN_THREADS), 0, s, (const ST_ *)x, n, partials);
    return hipGetLastError();
}

hipError_t normalize_impl(void *x, const void *buf1, size_t n, const DevState *st_, hipStream_t s) {
    hipLaunchKernelGGL(normalize_kernel<ST_>, dim3(1024), dim3(256), 0, s, (ST_ *)x, (const ST_ *)buf1, n, st_);
    return hipGetLastError();
}

hipError_t bound_impl(size_t n, const void *f, const void *x, uint32_t *out, hipStream_t s) {
    hipLaunchKernelGGL(bound_kernel<ST_>, dim3(1024), dim3(AUX_THREADS), 0, s, n, (const ST_ *)f,
                       (const ST_ *)x, out);
    return hipGetLastError();
}

hipError_t to_product_impl(const void *f, const void *x, void *buf1, size_t n, DevState *st_, hipStream_t s) {
    hipLaunchKernelGGL(to_product_kernel<ST_>, dim3(1024), dim3(256), 0, s, (const ST_ *)f, (const ST_ *)x,
                       (ST_ *)buf1, n, st_);
    return hipGetLastError();
}

hipError_t from_product_impl(void *x, const void *buf1, const void *f, size_t n, const DevState *st_, hipStream_t s) {
    hipLaunchKernelGGL(from_product_kernel<ST_>, dim3(1024), dim3(256), 0, s, (ST_ *)x, (const ST_ *)buf1,
                       (const ST_ *)f, n, st_);
    return hipGetLastError();
}

#define STPI_VARIANT_ENTRY(RS, RT, TH, TW, NTHR, RY, QX, OCC, PIPE) \
    {RS, RT, TH, TW, NTHR, RY, QX, OCC, PIPE, &launch_fwd<ST_, RS, RT, TH, TW, NTHR, RY, QX, OCC, PIPE>, \
     &fwd_blocks_per_cu<ST_, RS, RT, TH, TW, NTHR, RY, QX, OCC, PIPE>,                                 \
     product_launcher<ST_, RS, RT, TH, TW, NTHR, RY, QX, OCC, PIPE>()},

const Variant kVariants[] = {STPI_VARIANTS(STPI_VARIANT_ENTRY)};

#ifdef STPI_ADJ_VARIANTS
#define STPI_ADJ_ENTRY(RS, RT, TH, TW, NTHR, RY, QX) \
    {RS, RT, TH, TW, NTHR, RY, QX, &launch_adj<ST_, RS, RT, TH, TW, NTHR, RY, QX>},
const AdjVariant kAdj[] = {STPI_ADJ_VARIANTS(STPI_ADJ_ENTRY)};
constexpr int kNAdj = (int)(sizeof(kAdj) / sizeof(kAdj[0]));
#else
const AdjVariant *const kAdj = nullptr;
constexpr int kNAdj = 0;
#endif

hipError_t combine_fwd_impl(int C, size_t n, const void *fc, const double *w, void *f, hipStream_t s) {
    hipLaunchKernelGGL(combine_fwd_kernel<ST_>, dim3(1024), dim3(AUX_THREADS), 0, s, C, n, (const ST_ *)fc, w,
                       (ST_ *)f);
    return hipGetLastError();
}
hipError_t combine_bwd_impl(int C, size_t n, const void *fc, const void *gf, double *partials, hipStream_t s) {
    hipLaunchKernelGGL(combine_bwd_kernel<ST_>, dim3(AUX_BLOCKS), dim3(AUX_THREADS), 0, s, C, n, (const ST_ *)fc,
                       (const ST_ *)gf, partials);
    return hipGetLastError();
}
hipError_t scale_impl(size_t n, const void *z, const double *norm, void *x, hipStream_t s) {
    hipLaunchKernelGGL(scale_by_norm_kernel<ST_>, dim3(1024), dim3(AUX_THREADS), 0, s, n, (const ST_ *)z, norm,
                       (ST_ *)x);
    return hipGetLastError();
}
hipError_t dot_impl(size_t n, const void *a, const void *b, double *partials, hipStream_t s) {
    hipLaunchKernelGGL(dot_kernel<ST_>, dim3(AUX_BLOCKS), dim3(AUX_THREADS), 0, s, n, (const ST_ *)a,
                       (const ST_ *)b, partials);
    return hipGetLastError();
}
hipError_t train_init_impl(size_t n, void *x, double *norm, hipStream_t s) {
    hipLaunchKernelGGL(train_init_kernel<ST_>, dim3(1024), dim3(AUX_THREADS), 0, s, n, (ST_ *)x, norm);
    return hipGetLastError();
}
hipError_t max_impl(size_t n, const void *x, double *partials, hipStream_t s) {
    hipLaunchKernelGGL(max_kernel<ST_>, dim3(AUX_BLOCKS), dim3(AUX_THREADS), 0, s, n, (const ST_ *)x, partials);
    return hipGetLastError();
}
hipError_t bce_impl(size_t n, const void *x, const uint8_t *gt, const double *scalars, void *gx, double *partials,
                    hipStream_t s) {
    hipLaunchKernelGGL(bce_kernel<ST_>, dim3(AUX_BLOCKS), dim3(AUX_THREADS), 0, s, n, (const ST_ *)x, gt, scalars,
                       (ST_ *)gx, partials);
    return hipGetLastError();
}
hipError_t bce_fin_impl(size_t n, int nblocks, const double *partials, const double *scalars, void *gx,
                        double *loss, hipStream_t s) {
    hipLaunchKernelGGL(bce_finalize<ST_>, dim3(1), dim3(CHAIN_THREADS), 0, s, n, nblocks, partials, scalars,
                       (ST_ *)gx, loss);
    return hipGetLastError();
}

#ifdef STPI_BATCH_VARIANTS
#define STPI_BATCH_ENTRY(RS, RT, TH, TW, NTHR, RY, QX, PIPE)                                      \
    {RS, RT, TH, TW, NTHR, RY, QX, PIPE, &launch_batch<ST_, RS, RT, TH, TW, NTHR, RY, QX, PIPE>, \
     &batch_blocks_per_cu<ST_, RS, RT, TH, TW, NTHR, RY, QX, PIPE>},
const BatchVariant kBatch[] = {STPI_BATCH_VARIANTS(STPI_BATCH_ENTRY)};
constexpr int kNBatch = (int)(sizeof(kBatch) / sizeof(kBatch[0]));
#else
const BatchVariant *const kBatch = nullptr;
constexpr int kNBatch = 0;
#endif

hipError_t batch_fill_impl(void *x, const ClipDesc *clips, int nclips, hipStream_t s) {
    hipLaunchKernelGGL(batch_fill_ones_kernel<ST_>, dim3(BATCH_NORM_BLOCKS, nclips), dim3(256), 0, s, (ST_ *)x, clips);
    return hipGetLastError();
}
hipError_t batch_sumsq_impl(const void *x, const ClipDesc *clips, int nclips, double *partials, hipStream_t s) {
    hipLaunchKernelGGL(batch_sumsq_kernel<ST_>, dim3(BATCH_NORM_BLOCKS, nclips), dim3(256), 0, s, (const ST_ *)x,
                       clips, partials);
    return hipGetLastError();
}
hipError_t batch_normalize_impl(void *x, const void *buf1, const ClipDesc *clips, const DevState *states, int nclips,
                                hipStream_t s) {
    hipLaunchKernelGGL(batch_normalize_kernel<ST_>, dim3(BATCH_NORM_BLOCKS, nclips), dim3(256), 0, s, (ST_ *)x,
                       (const ST_ *)buf1, clips, states);
    return hipGetLastError();
}

hipError_t batch_bound_impl(const void *f, const ClipDesc *clips, DevState *states, int nclips, hipStream_t s) {
    hipLaunchKernelGGL(batch_bound_kernel<ST_>, dim3(BATCH_NORM_BLOCKS, nclips), dim3(256), 0, s, (const ST_ *)f,
                       clips, states);
    return hipGetLastError();
}
hipError_t batch_to_product_impl(const void *f, const void *x, void *buf1, const ClipDesc *clips, DevState *states,
                                 int nclips, hipStream_t s) {
    hipLaunchKernelGGL(batch_to_product_kernel<ST_>, dim3(BATCH_NORM_BLOCKS, nclips), dim3(256), 0, s,
                       (const ST_ *)f, (const ST_ *)x, (ST_ *)buf1, clips, states);
    return hipGetLastError();
}
hipError_t batch_from_product_impl(void *x, const void *buf1, const void *f, const ClipDesc *clips,
                                   const DevState *states, int nclips, hipStream_t s) {
    hipLaunchKernelGGL(batch_from_product_kernel<ST_>, dim3(BATCH_NORM_BLOCKS, nclips), dim3(256), 0, s, (ST_ *)x,
                       (const ST_ *)buf1, (const ST_ *)f, clips, states);
    return hipGetLastError();
}

hipError_t batch_refill_impl(void *x, void *buf1, const ClipDesc *clips, const DevState *states, int nclips,
                             hipStream_t s) {
    hipLaunchKernelGGL(batch_refill_kernel<ST_>, dim3(BATCH_NORM_BLOCKS, nclips), dim3(256), 0, s, (ST_ *)x,
                       (ST_ *)buf1, clips, states);
    return hipGetLastError();
}

const DtypeOps kOps = {sizeof(ST_),       kVariants,        (int)(sizeof(kVariants) / sizeof(kVariants[0])),
                       &fill_ones_impl,   &sumsq_impl,      &normalize_impl,
                       &bound_impl,        &to_product_impl, &from_product_impl,
                       kAdj,              kNAdj,            &combine_fwd_impl,
                       &combine_bwd_impl, &scale_impl,      &dot_impl,
                       &train_init_impl,  &max_impl,        &bce_impl,
                       &bce_fin_impl,     kBatch,           kNBatch,
                       &batch_fill_impl,  &batch_sumsq_impl, &batch_normalize_impl,
                       &batch_bound_impl, &batch_to_product_impl, &batch_from_product_impl,
                       &batch_refill_impl};

}  // namespace

const DtypeOps *STPI_NAME() { return &kOps; }

}  // namespace stpi
