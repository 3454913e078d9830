// Step kernels for FP16 deviation storage.
#include "lbm_step.h"

namespace clbm {
template struct StepKernels<1>;
}  // namespace clbm
