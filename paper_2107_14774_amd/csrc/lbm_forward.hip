// Forward entry points: the collide-and-stream step (kernels in lbm_step.h,
// one translation unit per storage type), initialisation, import/export of
// natural populations, observables with FP64 totals.
#include "lbm_internal.h"

namespace clbm {

// ------------------------------------------------------------------ init / import / export
// FP64 equilibrium deviation f_eq(rho, u) - w rho0 of one node, written
// without cancellation: d_rho E(x)E(x)E + rho0 [D(x)E(x)E + W0(x)D(x)E + W0(x)W0(x)D].
struct AxisD {
  double W0[3], E[3], D[3];
};

__device__ __forceinline__ AxisD axis_d(double u, int d, const ConstsD& kd) {
  AxisD v;
  const double q = u * u * kd.ic2[d], h = u * kd.ic[d];
  v.W0[0] = kd.w0s[d]; v.W0[1] = kd.w0c[d]; v.W0[2] = kd.w0s[d];
  v.D[0] = 0.5 * (q - h); v.D[1] = -q; v.D[2] = 0.5 * (q + h);
  for (int i = 0; i < 3; ++i) v.E[i] = v.W0[i] + v.D[i];
  return v;
}

__device__ __forceinline__ NodeCoord coord_of(int64_t node, const Consts& k) {
  const int x = (int)(node % k.nx);
  const int64_t t = node / k.nx;
  const int y = (int)(t % k.ny), z = (int)(t / k.ny);
  return make_coord(x, y, z, k);
}

template <int ST, int A = 0>
__device__ __forceinline__ void init_store(typename Store<ST>::T* __restrict__ dst, const NodeCoord& c,
                                           int64_t node, const AxisD& X, const AxisD& Y, const AxisD& Z,
                                           double drho, const double* __restrict__ perturb,
                                           const Consts& k, const ConstsD& kd) {
  constexpr int i = kEx[A] + 1, j = kEy[A] + 1, l = kEz[A] + 1;
  double v = drho * X.E[i] * Y.E[j] * Z.E[l]
           + kd.rho0 * (X.D[i] * Y.E[j] * Z.E[l] + X.W0[i] * Y.D[j] * Z.E[l] + X.W0[i] * Y.W0[j] * Z.D[l]);
  if (perturb != nullptr) v += perturb[A * k.n + node];
  dst[gather_slot<A>(c, k)] = Store<ST>::pack((float)(v * (double)k.sigma[wclass(A)]));
  if constexpr (A + 1 < 27) init_store<ST, A + 1>(dst, c, node, X, Y, Z, drho, perturb, k, kd);
}

template <int ST>
__global__ __launch_bounds__(256) void k_init(typename Store<ST>::T* __restrict__ dst,
                                              const double* __restrict__ rho, const double* __restrict__ u,
                                              const double* __restrict__ perturb, Consts k, ConstsD kd) {
  for (int64_t node = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; node < k.n;
       node += (int64_t)gridDim.x * blockDim.x) {
    const NodeCoord c = coord_of(node, k);
    const double rn = rho ? rho[node] : kd.rho0;
    const double ux = u ? u[node] : 0.0, uy = u ? u[k.n + node] : 0.0, uz = u ? u[2 * k.n + node] : 0.0;
    const AxisD X = axis_d(ux, 0, kd), Y = axis_d(uy, 1, kd), Z = axis_d(uz, 2, kd);
    init_store<ST>(dst, c, node, X, Y, Z, rn - kd.rho0, perturb, k, kd);
  }
}

template <int ST, int A = 0>
__device__ __forceinline__ void import_store(typename Store<ST>::T* __restrict__ dst, const NodeCoord& c,
                                             int64_t node, const double* __restrict__ f,
                                             const Consts& k, const ConstsD& kd) {
  const double v = f[A * k.n + node] - kd.w[A] * kd.rho0;
  dst[gather_slot<A>(c, k)] = Store<ST>::pack((float)(v * (double)k.sigma[wclass(A)]));
  if constexpr (A + 1 < 27) import_store<ST, A + 1>(dst, c, node, f, k, kd);
}

template <int ST>
__global__ __launch_bounds__(256) void k_import(typename Store<ST>::T* __restrict__ dst,
                                                const double* __restrict__ f, Consts k, ConstsD kd) {
  for (int64_t node = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; node < k.n;
       node += (int64_t)gridDim.x * blockDim.x) {
    import_store<ST>(dst, coord_of(node, k), node, f, k, kd);
  }
}

template <int ST, int A = 0>
__device__ __forceinline__ void export_load(const typename Store<ST>::T* __restrict__ src, const NodeCoord& c,
                                            int64_t node, double* __restrict__ f, const Consts& k,
                                            const ConstsD& kd) {
  const double v = (double)Store<ST>::load(src + gather_slot<A>(c, k)) / (double)k.sigma[wclass(A)];
  f[A * k.n + node] = kd.w[A] * kd.rho0 + v;
  if constexpr (A + 1 < 27) export_load<ST, A + 1>(src, c, node, f, k, kd);
}

template <int ST, int A = 0>
__device__ __forceinline__ void export_node(const typename Store<ST>::T* __restrict__ src, const NodeCoord& c,
                                            const Consts& k, const ConstsD& kd, double (&f)[27]) {
  f[A] = kd.w[A] * kd.rho0 + (double)Store<ST>::load(src + gather_slot<A>(c, k)) / (double)k.sigma[wclass(A)];
  if constexpr (A + 1 < 27) export_node<ST, A + 1>(src, c, k, kd, f);
}

template <int ST>
__global__ __launch_bounds__(256) void k_export(const typename Store<ST>::T* __restrict__ src,
                                                double* __restrict__ f, Consts k, ConstsD kd) {
  for (int64_t node = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; node < k.n;
       node += (int64_t)gridDim.x * blockDim.x) {
    export_load<ST>(src, coord_of(node, k), node, f, k, kd);
  }
}

// Natural populations of listed nodes (a sampled export): f[A][i] for node
// nodes[i]; an index outside [0, n) gives NaN for all 27 values.
template <int ST>
__global__ __launch_bounds__(256) void k_export_nodes(const typename Store<ST>::T* __restrict__ src,
                                                      const int64_t* __restrict__ nodes, int64_t count,
                                                      double* __restrict__ f, Consts k, ConstsD kd) {
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < count; i += (int64_t)gridDim.x * blockDim.x) {
    const int64_t node = nodes[i];
    if (node < 0 || node >= k.n) {
      for (int a = 0; a < 27; ++a) f[a * count + i] = __builtin_nan("");
      continue;
    }
    double tmp[27];
    const NodeCoord c = coord_of(node, k);
    export_node<ST>(src, c, k, kd, tmp);
    for (int a = 0; a < 27; ++a) f[a * count + i] = tmp[a];
  }
}

// ------------------------------------------------------------------ observables
__device__ __forceinline__ double wave_sum(double v) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
  return v;
}

__global__ void k_sums_reset(double* sums, double mass0) {
  if (threadIdx.x < 5) sums[threadIdx.x] = threadIdx.x == 0 ? mass0 : 0.0;
}

template <int ST>
__global__ __launch_bounds__(256) void k_moments(const typename Store<ST>::T* __restrict__ src,
                                                 const float* __restrict__ force, float* __restrict__ rho_out,
                                                 float* __restrict__ u_out, double* __restrict__ sums, Consts k) {
  double acc[5] = {0.0, 0.0, 0.0, 0.0, 0.0};
  for (int64_t node = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; node < k.n;
       node += (int64_t)gridDim.x * blockDim.x) {
    const NodeCoord c = coord_of(node, k);
    float df[27];
    gather_all<ST>(src, c, k, df);
    const LowMoments M = low_moments(df);
    float fx = k.fx, fy = k.fy, fz = k.fz;
    if (force != nullptr) {
      fx = force[node];
      fy = force[k.n + node];
      fz = force[2 * k.n + node];
    }
    const float rho = k.rho0 + M.m000;
    const float px = M.m100 + 0.5f * fx, py = k.r * M.m010 + 0.5f * fy, pz = k.s * M.m001 + 0.5f * fz;
    const float ux = px / rho, uy = py / rho, uz = pz / rho;
    if (rho_out) rho_out[node] = rho;
    if (u_out) {
      u_out[node] = ux;
      u_out[k.n + node] = uy;
      u_out[2 * k.n + node] = uz;
    }
    // totals from FP64 sums of the stored values (no FP32 rounding of the node sums)
    double dm = 0.0, dx = 0.0, dy = 0.0, dz = 0.0;
#pragma unroll
    for (int a = 0; a < 27; ++a) {
      const double v = (double)df[a];
      dm += v;
      if (kEx[a] != 0) dx += kEx[a] * v;
      if (kEy[a] != 0) dy += kEy[a] * v;
      if (kEz[a] != 0) dz += kEz[a] * v;
    }
    const double qx = dx + 0.5 * (double)fx, qy = (double)k.r * dy + 0.5 * (double)fy;
    const double qz = (double)k.s * dz + 0.5 * (double)fz;
    acc[0] += dm;
    acc[1] += qx;
    acc[2] += qy;
    acc[3] += qz;
    acc[4] += 0.5 * (qx * qx + qy * qy + qz * qz) / ((double)k.rho0 + dm);
  }
  if (sums == nullptr) return;
  __shared__ double part[5][4];
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
#pragma unroll
  for (int q = 0; q < 5; ++q) {
    const double v = wave_sum(acc[q]);
    if (lane == 0) part[q][wave] = v;
  }
  __syncthreads();
  if (threadIdx.x < 5) {
    const int nw = (blockDim.x + 63) / 64;
    double v = 0.0;
    for (int w = 0; w < nw; ++w) v += part[threadIdx.x][w];
    atomicAdd(&sums[threadIdx.x], v);
  }
}

// ------------------------------------------------------------------ launchers
static int grid_for(int64_t n, int block, int64_t cap) {
  int64_t g = (n + block - 1) / block;
  if (g > cap) g = cap;
  if (g < 1) g = 1;
  return (int)g;
}

hipError_t launch_step(const lbm_handle& h, const void* src, void* dst, const float* force,
                       const float* grad_src, float* drho_out, hipStream_t st) {
  switch (h.p.storage) {
    case LBM_F32: return StepKernels<0>::step(h, src, dst, force, grad_src, drho_out, st);
    case LBM_F16: return StepKernels<1>::step(h, src, dst, force, grad_src, drho_out, st);
    case LBM_BF16_SR: return StepKernels<3>::step(h, src, dst, force, grad_src, drho_out, st);
    default: return StepKernels<2>::step(h, src, dst, force, grad_src, drho_out, st);
  }
}

hipError_t launch_step_aa(const lbm_handle& h, void* state, int odd, const float* force, hipStream_t st) {
  switch (h.p.storage) {
    case LBM_F32: return StepKernels<0>::step_aa(h, state, odd, force, st);
    case LBM_F16: return StepKernels<1>::step_aa(h, state, odd, force, st);
    case LBM_BF16_SR: return StepKernels<3>::step_aa(h, state, odd, force, st);
    default: return StepKernels<2>::step_aa(h, state, odd, force, st);
  }
}

hipError_t launch_step_uniform(const lbm_handle& h, const void* src, void* dst, float fx, float fy, float fz,
                               hipStream_t st) {
  lbm_handle hv = h;  // host copy: the constants travel by value in the kernel arguments
  hv.k.fx = fx;
  hv.k.fy = fy;
  hv.k.fz = fz;
  return launch_step(hv, src, dst, nullptr, nullptr, nullptr, st);
}

hipError_t launch_step_aa_uniform(const lbm_handle& h, void* state, int odd, float fx, float fy, float fz,
                                  hipStream_t st) {
  lbm_handle hv = h;
  hv.k.fx = fx;
  hv.k.fy = fy;
  hv.k.fz = fz;
  return launch_step_aa(hv, state, odd, nullptr, st);
}

hipError_t launch_density(const lbm_handle& h, const void* src, float* drho, hipStream_t st) {
  switch (h.p.storage) {
    case LBM_F32: return StepKernels<0>::density(h, src, drho, st);
    case LBM_F16: return StepKernels<1>::density(h, src, drho, st);
    case LBM_BF16_SR: return StepKernels<3>::density(h, src, drho, st);
    default: return StepKernels<2>::density(h, src, drho, st);
  }
}

hipError_t launch_stream(const lbm_handle& h, const void* src, void* dst, hipStream_t st) {
  switch (h.p.storage) {
    case LBM_F32: return StepKernels<0>::stream(h, src, dst, st);
    case LBM_F16: return StepKernels<1>::stream(h, src, dst, st);
    case LBM_BF16_SR: return StepKernels<3>::stream(h, src, dst, st);
    default: return StepKernels<2>::stream(h, src, dst, st);
  }
}

// ------------------------------------------------------------------ plain copy
// One 16-byte non-temporal load and store per thread, no loop: of the copy
// shapes measured on 4-7 GB buffers this one moved the most bytes per second
// (a grid-stride loop of the same accesses ran about 20% slower).
typedef float f4_t __attribute__((ext_vector_type(4)));

__global__ __launch_bounds__(256) void k_copy16(const f4_t* __restrict__ src, f4_t* __restrict__ dst, uint64_t n16,
                                                uint64_t first) {
  const uint64_t i = first + (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n16) __builtin_nontemporal_store(__builtin_nontemporal_load(src + i), dst + i);
}

hipError_t launch_copy(void* dst, const void* src, size_t bytes, hipStream_t st) {
  const uint64_t n16 = bytes / 16;
  // launches of at most 2^31 - 1 blocks
  const uint64_t per_launch = (uint64_t)0x7fffffff * 256u;
  for (uint64_t first = 0; first < n16; first += per_launch) {
    const uint64_t cnt = n16 - first < per_launch ? n16 - first : per_launch;
    hipLaunchKernelGGL(k_copy16, (unsigned)((cnt + 255) / 256), 256, 0, st, (const f4_t*)src, (f4_t*)dst, n16, first);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
  }
  return hipSuccess;
}

hipError_t launch_init(const lbm_handle& h, void* dst, const double* rho, const double* u,
                       const double* perturb, hipStream_t st) {
  const int g = grid_for(h.n, 256, 65536);
  switch (h.p.storage) {
    case LBM_F32: hipLaunchKernelGGL(k_init<0>, g, 256, 0, st, (float*)dst, rho, u, perturb, h.k, h.kd); break;
    case LBM_F16: hipLaunchKernelGGL(k_init<1>, g, 256, 0, st, (Store<1>::T*)dst, rho, u, perturb, h.k, h.kd); break;
    default: hipLaunchKernelGGL(k_init<2>, g, 256, 0, st, (Store<2>::T*)dst, rho, u, perturb, h.k, h.kd); break;
  }
  return hipGetLastError();
}

hipError_t launch_import(const lbm_handle& h, void* dst, const double* f, hipStream_t st) {
  const int g = grid_for(h.n, 256, 65536);
  switch (h.p.storage) {
    case LBM_F32: hipLaunchKernelGGL(k_import<0>, g, 256, 0, st, (float*)dst, f, h.k, h.kd); break;
    case LBM_F16: hipLaunchKernelGGL(k_import<1>, g, 256, 0, st, (Store<1>::T*)dst, f, h.k, h.kd); break;
    default: hipLaunchKernelGGL(k_import<2>, g, 256, 0, st, (Store<2>::T*)dst, f, h.k, h.kd); break;
  }
  return hipGetLastError();
}

hipError_t launch_export(const lbm_handle& h, const void* src, double* f, hipStream_t st) {
  const int g = grid_for(h.n, 256, 65536);
  switch (h.p.storage) {
    case LBM_F32: hipLaunchKernelGGL(k_export<0>, g, 256, 0, st, (const float*)src, f, h.k, h.kd); break;
    case LBM_F16: hipLaunchKernelGGL(k_export<1>, g, 256, 0, st, (const Store<1>::T*)src, f, h.k, h.kd); break;
    default: hipLaunchKernelGGL(k_export<2>, g, 256, 0, st, (const Store<2>::T*)src, f, h.k, h.kd); break;
  }
  return hipGetLastError();
}

hipError_t launch_export_nodes(const lbm_handle& h, const void* src, const int64_t* nodes, int64_t count, double* f,
                              hipStream_t st) {
  if (count == 0) return hipSuccess;
  const int g = grid_for(count, 256, 65536);
  switch (h.p.storage) {
    case LBM_F32:
      hipLaunchKernelGGL(k_export_nodes<0>, g, 256, 0, st, (const float*)src, nodes, count, f, h.k, h.kd);
      break;
    case LBM_F16:
      hipLaunchKernelGGL(k_export_nodes<1>, g, 256, 0, st, (const Store<1>::T*)src, nodes, count, f, h.k, h.kd);
      break;
    default:
      hipLaunchKernelGGL(k_export_nodes<2>, g, 256, 0, st, (const Store<2>::T*)src, nodes, count, f, h.k, h.kd);
      break;
  }
  return hipGetLastError();
}

hipError_t launch_moments(const lbm_handle& h, const void* src, const float* force, float* rho,
                          float* u, double* sums, hipStream_t st) {
  if (sums) {
    hipLaunchKernelGGL(k_sums_reset, 1, 64, 0, st, sums, (double)h.n * h.kd.rho0);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
  }
  const int g = grid_for(h.n, 256, 4096);
  switch (h.p.storage) {
    case LBM_F32: hipLaunchKernelGGL(k_moments<0>, g, 256, 0, st, (const float*)src, force, rho, u, sums, h.k); break;
    case LBM_F16: hipLaunchKernelGGL(k_moments<1>, g, 256, 0, st, (const Store<1>::T*)src, force, rho, u, sums, h.k); break;
    default: hipLaunchKernelGGL(k_moments<2>, g, 256, 0, st, (const Store<2>::T*)src, force, rho, u, sums, h.k); break;
  }
  return hipGetLastError();
}

}  // namespace clbm
