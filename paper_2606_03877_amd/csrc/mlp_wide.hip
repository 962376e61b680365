// Forward kernels of the networks wider than 64 (Sec. 3.2), compiled as a
// unit of their own so that they keep the compiler's default assignment of
// matrix-core accumulators.
#define MSPLAT_WIDE_TU
#include "mlp.hip"
