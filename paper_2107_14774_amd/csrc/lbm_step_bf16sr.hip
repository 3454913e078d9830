// Step kernels for BF16 deviation storage with stochastic rounding.
#include "lbm_step.h"

namespace clbm {
template struct StepKernels<3>;
}  // namespace clbm
