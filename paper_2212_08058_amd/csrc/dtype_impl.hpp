// Instantiates the kernel set for one storage type. Included once per type by
// kernels_<type>.hip with STPI_ST (storage type), STPI_NAME (suffix) and
// STPI_VARIANTS(X) (the compiled (RS, RT, TH, TW, NTHR, RY) list) defined.
#pragma once

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

#define STPI_VARIANT_ENTRY(RS, RT, TH, TW, NTHR, RY) \
    {RS, RT, TH, TW, NTHR, RY, &launch_fwd<ST_, RS, RT, TH, TW, NTHR, RY>},

const Variant kVariants[] = {STPI_VARIANTS(STPI_VARIANT_ENTRY)};

const DtypeOps kOps = {sizeof(ST_), kVariants, (int)(sizeof(kVariants) / sizeof(kVariants[0])),
                       &fill_ones_impl, &sumsq_impl, &normalize_impl};

}  // namespace

const DtypeOps *STPI_NAME() { return &kOps; }

}  // namespace stpi
