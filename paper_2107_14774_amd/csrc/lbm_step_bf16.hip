// Step kernels for BF16 deviation storage.
#include "lbm_step.h"

namespace clbm {
template struct StepKernels<2>;
}  // namespace clbm
