// Adjoint step kernels for BF16 deviation storage.
#include "lbm_adjoint_step.h"

namespace clbm {
template struct AdjointKernels<2>;
}  // namespace clbm
