// Kernel set with bfloat16 storage (round to nearest even on store) and float arithmetic.
#include "common.hpp"
#define STPI_ST ::stpi::bf16
#define STPI_NAME dtype_ops_bf16
#define STPI_VARIANTS(X)            \
    X(1, 1, 16, 64, 256, 8, 4, 1)      \
    X(2, 1, 16, 64, 256, 8, 4, 1)      \
    X(2, 2, 16, 64, 256, 8, 4, 1)      \
    X(4, 2, 16, 64, 256, 8, 4, 1)      \
    X(8, 3, 16, 64, 256, 8, 4, 1)      \
    X(8, 3, 8, 128, 256, 8, 4, 1)      \
    X(8, 3, 8, 64, 128, 8, 4, 1)       \
    X(8, 8, 16, 64, 256, 8, 4, 1)      \
    X(15, 5, 16, 64, 256, 8, 4, 1)     \
    X(15, 5, 8, 128, 256, 8, 4, 1)     \
    X(15, 5, 16, 64, 256, 8, 4, 3)     \
    X(15, 5, 8, 128, 256, 8, 4, 3)     \
    X(16, 8, 16, 64, 256, 8, 4, 3)     \
    X(15, 5, 8, 64, 128, 8, 4, 1)      \
    X(15, 5, 16, 128, 512, 8, 4, 1)    \
    X(16, 8, 16, 64, 256, 8, 4, 1)
#define STPI_BATCH_VARIANTS(X)       \
    X(8, 3, 16, 64, 256, 8, 4)   \
    X(8, 3, 8, 64, 128, 8, 4)    \
    X(16, 8, 16, 64, 256, 8, 4)
#include "dtype_impl.hpp"
