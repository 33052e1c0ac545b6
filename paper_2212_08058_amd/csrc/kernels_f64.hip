// Kernel set with double storage and arithmetic (gradient and oracle-precision checks).
#include "common.hpp"
#define STPI_ST double
#define STPI_NAME dtype_ops_f64
#define STPI_VARIANTS(X)            \
    X(1, 1, 16, 64, 256, 8, 4, 1, 0)      \
    X(2, 1, 16, 64, 256, 8, 4, 1, 0)      \
    X(2, 2, 16, 64, 256, 8, 4, 1, 0)      \
    X(4, 2, 16, 64, 256, 8, 4, 1, 0)      \
    X(4, 2, 16, 64, 256, 8, 4, 1, 1)      \
    X(8, 3, 16, 64, 256, 8, 4, 1, 0)      \
    X(8, 8, 16, 64, 256, 8, 4, 1, 0)      \
    X(16, 8, 16, 64, 256, 8, 4, 1, 0)
#define STPI_ADJ_VARIANTS(X)     \
    X(1, 1, 16, 64, 256, 8, 4)   \
    X(2, 2, 16, 64, 256, 8, 4)   \
    X(4, 2, 16, 64, 256, 8, 4)   \
    X(8, 3, 16, 64, 256, 8, 4)   \
    X(16, 8, 16, 64, 256, 8, 4)
#define STPI_BATCH_VARIANTS(X)       \
    X(4, 2, 16, 64, 256, 8, 4, 0)   \
    X(16, 8, 16, 64, 256, 8, 4, 0)
#include "dtype_impl.hpp"
