// Host-side handle and kernel launchers shared by the translation units of
// the library (not part of the public C ABI).
#pragma once

#include <hip/hip_runtime.h>

#include "../../include/lbm.h"
#include "lbm_device.h"

struct lbm_handle {
  lbm_params p;
  clbm::Consts k;
  clbm::ConstsD kd;
  int64_t n;         // nodes
  int64_t stride;    // slots per direction: nodes with every x-row padded to a multiple of clbm::kB
  size_t elem;       // bytes per stored element
  size_t bytes;      // bytes of one state (27 stride elem)
  int block;         // threads per block of the node kernels
  int block_step;    // threads per block of the FP32 step without full corrections
  int pairs;         // 1 = the periodic 16-bit step may run two nodes per thread
  int step_lds;      // dynamic LDS bytes per block of the one-node steps without full
                     // corrections, AB and AA (unused by the kernels; caps the blocks per CU)
  int pair_lds;      // the same for the 16-bit steps with two nodes per thread (AB and AA)
  uint64_t seq;      // step counter: keys the stochastic rounding of BF16-SR storage
  int force_kind;    // 0, or a more general gather path to take where valid (1: 32-bit
                     // offsets across the state, 2: 64-bit slots); a testing override
};

namespace clbm {

// Step and adjoint-step launchers per storage type (0 FP32, 1 FP16, 2 BF16,
// 3 BF16 with stochastic rounding, whose adjoint reads the state like 2); each
// is instantiated in a translation unit of its own.
template <int ST>
struct StepKernels {
  static hipError_t step(const lbm_handle& h, const void* src, void* dst, const float* force,
                         const float* grad_src, float* drho_out, hipStream_t st);
  static hipError_t step_aa(const lbm_handle& h, void* state, int odd, const float* force, hipStream_t st);
  static hipError_t density(const lbm_handle& h, const void* src, float* drho, hipStream_t st);
  static hipError_t stream(const lbm_handle& h, const void* src, void* dst, hipStream_t st);
};
extern template struct StepKernels<0>;
extern template struct StepKernels<1>;
extern template struct StepKernels<2>;
extern template struct StepKernels<3>;

template <int ST>
struct AdjointKernels {
  // drho, grad_rho: the full corrections' density field of the state and the field that receives
  // the cotangent of its gradient (NULL otherwise); pend: grad_rho's first component holds on entry a
  // per-node value to add to each of the node's 27 outputs
  static hipError_t step(const lbm_handle& h, const void* state, const float* adj_in, float* adj_out,
                         const float* force, float* grad_force, double* grad_uniform, const float* drho,
                         float* grad_rho, bool pend, hipStream_t st);
  // the data movement of step (local corrections) without its arithmetic
  static hipError_t stream(const lbm_handle& h, const void* state, const float* adj_in, float* adj_out,
                           const float* force, float* grad_force, hipStream_t st);
};
extern template struct AdjointKernels<0>;
extern template struct AdjointKernels<1>;
extern template struct AdjointKernels<2>;

hipError_t launch_step(const lbm_handle& h, const void* src, void* dst, const float* force,
                       const float* grad_src, float* drho_out, hipStream_t st);
// Same with the uniform force replaced for this launch only.
hipError_t launch_step_uniform(const lbm_handle& h, const void* src, void* dst, float fx, float fy, float fz,
                               hipStream_t st);
hipError_t launch_density(const lbm_handle& h, const void* src, float* drho, hipStream_t st);
// Streaming only (the step without its collision).
hipError_t launch_stream(const lbm_handle& h, const void* src, void* dst, hipStream_t st);
// Plain device copy, one 16-byte load and store per thread.
hipError_t launch_copy(void* dst, const void* src, size_t bytes, hipStream_t st);
// AA layout: one step in place; odd selects the shifted half of the pair.
hipError_t launch_step_aa(const lbm_handle& h, void* state, int odd, const float* force, hipStream_t st);
hipError_t launch_step_aa_uniform(const lbm_handle& h, void* state, int odd, float fx, float fy, float fz,
                                  hipStream_t st);
hipError_t launch_init(const lbm_handle& h, void* dst, const double* rho, const double* u,
                       const double* perturb, hipStream_t st);
hipError_t launch_import(const lbm_handle& h, void* dst, const double* f, hipStream_t st);
hipError_t launch_export(const lbm_handle& h, const void* src, double* f, hipStream_t st);
hipError_t launch_export_nodes(const lbm_handle& h, const void* src, const int64_t* nodes, int64_t count, double* f,
                              hipStream_t st);
hipError_t launch_moments(const lbm_handle& h, const void* src, const float* force, float* rho,
                          float* u, double* sums, hipStream_t st);
// With the full corrections drho (float[n]) and grad_rho (float[3 n]) are the caller's fields:
// exact = true adds the gradient's transpose to adj_out and computes drho from the state unless
// drho_given; else drho is read, and pending (float[3 n] or NULL) is a cotangent whose transpose is
// added to adj_out.
hipError_t launch_step_adjoint(const lbm_handle& h, const void* state, const float* adj_in,
                               float* adj_out, const float* force, float* grad_force,
                               double* grad_force_uniform, float* drho, float* grad_rho, bool exact,
                               bool drho_given, const float* pending, hipStream_t st);
// adj += the density-gradient stencil's transpose of grad (full corrections)
hipError_t launch_density_adjoint(const lbm_handle& h, const float* grad, float* adj, hipStream_t st);
hipError_t launch_moments_adjoint(const lbm_handle& h, const void* state, const float* force,
                                  const float* g_rho, const float* g_u, float* adj,
                                  float* grad_force, hipStream_t st);
hipError_t launch_init_adjoint(const lbm_handle& h, const float* adj, const double* rho,
                               const double* u, double* g_rho, double* g_u, hipStream_t st);
hipError_t launch_adjoint_natural(const lbm_handle& h, const float* slots, double* natural,
                                  int to_natural, const double* natural_in, float* slots_out,
                                  hipStream_t st);

}  // namespace clbm
