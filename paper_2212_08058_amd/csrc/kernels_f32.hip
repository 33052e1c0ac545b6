// Kernel set with float storage and float arithmetic.
#include "common.hpp"
#define STPI_ST float
#define STPI_NAME dtype_ops_f32
#define STPI_VARIANTS(X)            \
    X(1, 1, 16, 64, 256, 4)         \
    X(2, 1, 16, 64, 256, 4)         \
    X(2, 2, 16, 64, 256, 4)         \
    X(4, 2, 16, 64, 256, 4)         \
    X(8, 3, 16, 64, 256, 8)         \
    X(8, 3, 16, 128, 256, 16)       \
    X(8, 8, 16, 64, 256, 8)         \
    X(15, 5, 16, 64, 256, 8)      \
    X(16, 8, 16, 64, 256, 8)
#include "dtype_impl.hpp"
