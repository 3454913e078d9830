// Adjoint step kernels for FP16 deviation storage.
#include "lbm_adjoint_step.h"

namespace clbm {
template struct AdjointKernels<1>;
}  // namespace clbm
