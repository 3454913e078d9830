// Step kernels for FP32 storage.
#include "lbm_step.h"

namespace clbm {
template struct StepKernels<0>;
}  // namespace clbm
