// Per-storage-type entry points of the kernel set (one translation unit per type).
#pragma once

#include "forward.hpp"

namespace stpi {

struct DtypeOps {
    size_t elem;                 // bytes per stored element
    const Variant *variants;     // compiled step kernels
    int nvariants;
    hipError_t (*fill_ones)(void *x, size_t n, hipStream_t);
    hipError_t (*sumsq)(const void *x, size_t n, double *partials, hipStream_t);
    hipError_t (*normalize)(void *x, const void *buf1, size_t n, const DevState *s, hipStream_t);
};

const DtypeOps *dtype_ops_f32();
const DtypeOps *dtype_ops_bf16();
const DtypeOps *dtype_ops_f64();

}  // namespace stpi
