// Adjoint step kernels for FP32 storage.
#include "lbm_adjoint_step.h"

namespace clbm {
template struct AdjointKernels<0>;
}  // namespace clbm
