// Backward kernels of the networks wider than 64, compiled as a unit of their
// own (see mlp_wide.hip).
#define MSPLAT_WIDE_TU
#include "mlp_bwd.hip"
