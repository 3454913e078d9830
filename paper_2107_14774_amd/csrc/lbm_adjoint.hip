// Adjoint kernels (reverse mode of the fused step and of its two ends).
#include "lbm_internal.h"

namespace clbm {

hipError_t launch_step_adjoint(const lbm_handle&, const void*, const float*, float*, const float*, float*,
                               double*, hipStream_t) {
  return hipErrorNotSupported;
}
hipError_t launch_moments_adjoint(const lbm_handle&, const void*, const float*, const float*, const float*,
                                  float*, float*, hipStream_t) {
  return hipErrorNotSupported;
}
hipError_t launch_init_adjoint(const lbm_handle&, const float*, const double*, const double*, double*, double*,
                               hipStream_t) {
  return hipErrorNotSupported;
}
hipError_t launch_adjoint_natural(const lbm_handle&, const float*, double*, int, const double*, float*,
                                  hipStream_t) {
  return hipErrorNotSupported;
}

}  // namespace clbm
