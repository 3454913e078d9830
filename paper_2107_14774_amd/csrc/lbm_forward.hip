// Forward kernels: fused collide-and-stream step, initialisation,
// import/export of natural populations, observables with FP64 totals.
#include "lbm_internal.h"

namespace clbm {

// ------------------------------------------------------------------ step
// One thread per node, pull scheme: gather 27 slots of the source buffer,
// collide, write the node's 27 slots of the destination buffer (coalesced
// along x, non-temporal).  Without walls every source slot is
// (alpha, x - ebar_alpha) with periodic wrap, addressed as a per-direction
// base pointer plus a 32-bit node index shared by the three directions of
// one source row; with walls the general slot rule of gather_slot applies.
// With the full corrections (CORR 3) the density gradient comes from the
// density-deviation field grad_src, and drho_out (if not NULL) receives the
// node's own density deviation.
// WALLS: 0 periodic (per-direction bases, 32-bit offsets), 1 walls with 32-bit
// offsets from direction 0's array (state below 4 GiB), 2 walls, 64-bit slots.
template <int ST, int WALLS>
__device__ __forceinline__ void gather_node(const DirPtrs<typename Store<ST>::T>& P, int x, int y, int z,
                                            const Consts& k, float (&df)[27]) {
  if constexpr (WALLS == 2) {
    gather_all<ST>(P.src[0], make_coord(x, y, z, k), k, df);
  } else {
    PeriodicRows pr;
    periodic_rows(x, y, z, k, pr);
    if constexpr (WALLS == 1) {
      const uint32_t node = ((uint32_t)z * (uint32_t)k.ny + (uint32_t)y) * (uint32_t)k.nx + (uint32_t)x;
      gather_walls32<ST>(P.src[0], pr, node, wall_flags(x, y, z, k), k, df);
    } else {
      gather_periodic<ST>(P.src, pr, k, df);
    }
  }
}

// Minimum waves per SIMD the compiler must fit (1 = no register limit).
#ifndef LBM_STEP_WAVES_F32
#define LBM_STEP_WAVES_F32 1
#endif
#ifndef LBM_STEP_WAVES_F16
#define LBM_STEP_WAVES_F16 1
#endif
#ifndef LBM_FULL_WAVES_F32
#define LBM_FULL_WAVES_F32 1
#endif
#ifndef LBM_FULL_WAVES_F16
#define LBM_FULL_WAVES_F16 1
#endif
constexpr int step_waves(int st, int corr) {
  return corr == 3 ? (st == 0 ? LBM_FULL_WAVES_F32 : LBM_FULL_WAVES_F16)
                   : (st == 0 ? LBM_STEP_WAVES_F32 : LBM_STEP_WAVES_F16);
}

template <int ST, int CORR, int WALLS, bool RAW>
__global__ __launch_bounds__(256, step_waves(ST, CORR)) void k_step(DirPtrs<typename Store<ST>::T> P,
                                              const float* __restrict__ force,
                                              const float* __restrict__ grad_src, float* __restrict__ drho_out,
                                              Consts k, uint32_t bpr) {
  const uint32_t lb = xcd_block(blockIdx.x, gridDim.x);
  const uint32_t bxi = lb % bpr, rowid = lb / bpr;
  int y, z;
  if constexpr (CORR == 3) {
    // rows in y-tiles of k.ytile, z-major inside a tile: the density rows of z - 1 and
    // z + 1 are then read a few rows apart (an L2 hit) instead of a whole plane apart
    const uint32_t ty = (uint32_t)k.ytile, per_tile = ty * (uint32_t)k.nz;
    const uint32_t tile = rowid / per_tile, rem = rowid % per_tile;
    z = (int)(rem / ty);
    y = (int)(tile * ty + rem % ty);
  } else {
    y = (int)(rowid % (uint32_t)k.ny);
    z = (int)(rowid / (uint32_t)k.ny);
  }
  const int x = (int)(bxi * blockDim.x + threadIdx.x);
  // the density gradient first (block-wide, with a barrier), while no population is live
  float grx = 0.0f, gry = 0.0f, grz = 0.0f;
  if constexpr (CORR == 3) {
    __shared__ float lds[3][258];
    density_gradient_block(grad_src, x, y, z, x < k.nx, k, lds, grx, gry, grz);
  }
  if (x >= k.nx) return;
  const uint32_t node = ((uint32_t)z * (uint32_t)k.ny + (uint32_t)y) * (uint32_t)k.nx + (uint32_t)x;
  float df[27];
  gather_node<ST, WALLS>(P, x, y, z, k, df);
  float fx = k.fx, fy = k.fy, fz = k.fz;
  if (force != nullptr) {
    fx = ld_off(force, node);
    fy = ld_off(force + k.n, node);
    fz = ld_off(force + 2 * k.n, node);
  }
  float out[27];
  if constexpr (CORR == 3) {
    collide_node<CORR, RAW>(df, fx, fy, fz, k, out, grx, gry, grz);
    if (drho_out != nullptr) drho_out[node] = low_moments(df).m000;
  } else {
    collide_node<CORR, RAW>(df, fx, fy, fz, k, out);
  }
  if constexpr (ST == 0) conserve(df, fx, fy, fz, k, out);
  if constexpr (WALLS != 0) {
    if (k.moving) moving_wall_terms(x, y, z, k.rho0 + low_moments(df).m000, k, out);
  }
#pragma unroll
  for (int a = 0; a < 27; ++a)
    st_off_nt(P.dst[a], node, Store<ST>::pack(ST == 0 ? out[a] : out[a] * k.sigma[a]));
}

// ------------------------------------------------------------------ step, AA layout
// One buffer updated in place.  Even steps (ODD = false): node x reads its own
// slots (a, x), collides and writes f~_a to (opp(a), x).  Odd steps: f_a(x) is
// read from (opp(a), x - ebar_a), or from (a, x) when x - ebar_a lies beyond a
// wall, and f~_a is written to (a, x + ebar_a), or to (opp(a), x) when
// x + ebar_a lies beyond a wall.  Within a step every slot is read and written
// by one node only, so the update needs no second buffer.  After an even
// number of steps slot (a, x) holds f_a(x) again.  Without walls each direction
// array is addressed through its own base pointer; with walls all 27 arrays
// through direction 0's base with 32-bit offsets (the state below 4 GiB).
template <int A>
__device__ __forceinline__ bool pulls_through_wall(const WallFlags& w) {
  constexpr int ex = kEx[A], ey = kEy[A], ez = kEz[A];
  bool wall = false;
  if (ex > 0) wall |= w.lx;
  if (ex < 0) wall |= w.hx;
  if (ey > 0) wall |= w.ly;
  if (ey < 0) wall |= w.hy;
  if (ez > 0) wall |= w.lz;
  if (ez < 0) wall |= w.hz;
  return wall;
}

template <int ST, bool ODD, bool WALLS, int A = 0>
__device__ __forceinline__ void gather_aa(const DirPtrs<typename Store<ST>::T>& P, const PeriodicRows& pr, uint32_t node,
                                          const WallFlags& w, const Consts& k, float (&df)[27]) {
  constexpr int opp = opposite_of(A);
  typename Store<ST>::T v;
  if constexpr (!ODD) {
    v = ld_off(P.src[A], node);
  } else if constexpr (WALLS) {
    const uint32_t stride = (uint32_t)k.stride;
    const uint32_t idx = pulls_through_wall<A>(w) ? (uint32_t)A * stride + node
                                                  : (uint32_t)opp * stride + periodic_src<A>(pr);
    v = ld_off(P.src[0], idx);
  } else {
    v = ld_off(P.src[opp], periodic_src<A>(pr));
  }
  const float f = Store<ST>::load_val(v);
  df[A] = ST == 0 ? f : f * k.inv_sigma[A];
  if constexpr (A + 1 < 27) gather_aa<ST, ODD, WALLS, A + 1>(P, pr, node, w, k, df);
}

template <typename T>
__device__ __forceinline__ void st_off(T* __restrict__ base, uint32_t idx, T v) {
  *reinterpret_cast<T*>(reinterpret_cast<char*>(base) + (uint32_t)(idx * (uint32_t)sizeof(T))) = v;
}

template <int ST, bool ODD, bool WALLS, int A = 0>
__device__ __forceinline__ void store_aa(const DirPtrs<typename Store<ST>::T>& P, const PeriodicRows& pr, uint32_t node,
                                         const WallFlags& w, const Consts& k, const float (&out)[27]) {
  constexpr int opp = opposite_of(A);
  const typename Store<ST>::T v = Store<ST>::pack(ST == 0 ? out[A] : out[A] * k.sigma[A]);
  if constexpr (!ODD) {
    st_off_nt(P.dst[opp], node, v);
  } else if constexpr (WALLS) {
    // x + ebar_A lies beyond a wall exactly when opp(A) pulls through one
    const uint32_t stride = (uint32_t)k.stride;
    const uint32_t idx = pulls_through_wall<opp>(w) ? (uint32_t)opp * stride + node
                                                    : (uint32_t)A * stride + periodic_src<opp>(pr);
    st_off(P.dst[0], idx, v);
  } else {
    // shifted by one node along x for most directions: plain stores, partial lines merge in L2
    // (non-temporal stores measured 0-1.5% slower here)
    st_off(P.dst[A], periodic_src<opp>(pr), v);
  }
  if constexpr (A + 1 < 27) store_aa<ST, ODD, WALLS, A + 1>(P, pr, node, w, k, out);
}

template <int ST, int CORR, bool ODD, bool WALLS, bool RAW>
__global__ __launch_bounds__(256, step_waves(ST, CORR)) void k_step_aa(DirPtrs<typename Store<ST>::T> P,
                                                                       const float* __restrict__ force, Consts k,
                                                                       uint32_t bpr) {
  const uint32_t lb = xcd_block(blockIdx.x, gridDim.x);
  const uint32_t bxi = lb % bpr, rowid = lb / bpr;
  const int y = (int)(rowid % (uint32_t)k.ny), z = (int)(rowid / (uint32_t)k.ny);
  const int x = (int)(bxi * blockDim.x + threadIdx.x);
  if (x >= k.nx) return;
  const uint32_t node = ((uint32_t)z * (uint32_t)k.ny + (uint32_t)y) * (uint32_t)k.nx + (uint32_t)x;
  PeriodicRows pr;
  WallFlags w{};
  if constexpr (ODD) periodic_rows(x, y, z, k, pr);
  if constexpr (WALLS) w = wall_flags(x, y, z, k);
  float df[27];
  gather_aa<ST, ODD, WALLS>(P, pr, node, w, k, df);
  float fx = k.fx, fy = k.fy, fz = k.fz;
  if (force != nullptr) {
    fx = ld_off(force, node);
    fy = ld_off(force + k.n, node);
    fz = ld_off(force + 2 * k.n, node);
  }
  float out[27];
  collide_node<CORR, RAW>(df, fx, fy, fz, k, out);
  if constexpr (ST == 0) conserve(df, fx, fy, fz, k, out);
  if constexpr (WALLS) {
    if (k.moving) moving_wall_terms(x, y, z, k.rho0 + low_moments(df).m000, k, out);
  }
  store_aa<ST, ODD, WALLS>(P, pr, node, w, k, out);
}

// Density deviation of every node of a state: the same gather and the same
// FP32 sum as the step, so the value is bit-identical to the step's.
template <int ST, int WALLS>
__global__ __launch_bounds__(256) void k_density(DirPtrs<typename Store<ST>::T> P, float* __restrict__ drho,
                                                 Consts k, uint32_t bpr) {
  const uint32_t lb = xcd_block(blockIdx.x, gridDim.x);
  const uint32_t bxi = lb % bpr, rowid = lb / bpr;
  const int y = (int)(rowid % (uint32_t)k.ny), z = (int)(rowid / (uint32_t)k.ny);
  const int x = (int)(bxi * blockDim.x + threadIdx.x);
  if (x >= k.nx) return;
  const uint32_t node = ((uint32_t)z * (uint32_t)k.ny + (uint32_t)y) * (uint32_t)k.nx + (uint32_t)x;
  float df[27];
  gather_node<ST, WALLS>(P, x, y, z, k, df);
  drho[node] = low_moments(df).m000;
}

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
  dst[gather_slot<A>(c, k)] = Store<ST>::pack((float)(v * (double)k.sigma[A]));
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
  dst[gather_slot<A>(c, k)] = Store<ST>::pack((float)(v * (double)k.sigma[A]));
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
  const double v = (double)Store<ST>::load(src + gather_slot<A>(c, k)) / (double)k.sigma[A];
  f[A * k.n + node] = kd.w[A] * kd.rho0 + v;
  if constexpr (A + 1 < 27) export_load<ST, A + 1>(src, c, node, f, k, kd);
}

template <int ST>
__global__ __launch_bounds__(256) void k_export(const typename Store<ST>::T* __restrict__ src,
                                                double* __restrict__ f, Consts k, ConstsD kd) {
  for (int64_t node = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; node < k.n;
       node += (int64_t)gridDim.x * blockDim.x) {
    export_load<ST>(src, coord_of(node, k), node, f, k, kd);
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
// Gather path: 0 periodic (32-bit offsets per direction array), 1 walls with
// 32-bit offsets across the whole state, 2 walls with 64-bit slots.
static int gather_kind(const lbm_handle& h) {
  const bool walls = h.k.bb_x || h.k.bb_y || h.k.bb_z;
  if (!walls && (uint64_t)h.stride * h.elem < (1ull << 32)) return 0;
  if (27ull * (uint64_t)h.stride * h.elem < (1ull << 32)) return 1;
  return 2;
}

static int grid_for(int64_t n, int block, int64_t cap) {
  int64_t g = (n + block - 1) / block;
  if (g > cap) g = cap;
  if (g < 1) g = 1;
  return (int)g;
}

template <int ST>
static hipError_t launch_step_t(const lbm_handle& h, const void* src, void* dst, const float* force,
                                const float* grad_src, float* drho_out, hipStream_t st) {
  using T = typename Store<ST>::T;
  const int block = h.block;
  const uint32_t bpr = (uint32_t)((h.p.nx + block - 1) / block);
  const int64_t nb = (int64_t)bpr * h.p.ny * h.p.nz;
  if (nb > 0x7fffffffLL) return hipErrorInvalidConfiguration;
  DirPtrs<T> P;
  for (int a = 0; a < 27; ++a) {
    P.src[a] = (const T*)src + (int64_t)a * h.stride;
    P.dst[a] = (T*)dst + (int64_t)a * h.stride;
  }
  const int kind = gather_kind(h);
  const dim3 grid((unsigned)nb), blk(block);
#define CLBM_STEP(C, W, R) \
  hipLaunchKernelGGL((k_step<ST, C, W, R>), grid, blk, 0, st, P, force, grad_src, drho_out, h.k, bpr)
#define CLBM_STEP_CORR(W, R)                   \
  switch (h.p.corr) {                          \
    case 0: CLBM_STEP(0, W, R); break;         \
    case 1: CLBM_STEP(1, W, R); break;         \
    case 2: CLBM_STEP(2, W, R); break;         \
    default: CLBM_STEP(3, W, R); break;        \
  }
#define CLBM_STEP_RAW(W)                                           \
  if (h.p.moments == LBM_RAW) { CLBM_STEP_CORR(W, true) } else { CLBM_STEP_CORR(W, false) }
  if (kind == 0) {
    CLBM_STEP_RAW(0)
  } else if (kind == 1) {
    CLBM_STEP_RAW(1)
  } else {
    CLBM_STEP_RAW(2)
  }
#undef CLBM_STEP_RAW
#undef CLBM_STEP_CORR
#undef CLBM_STEP
  return hipGetLastError();
}

template <int ST>
static hipError_t launch_density_t(const lbm_handle& h, const void* src, float* drho, hipStream_t st) {
  using T = typename Store<ST>::T;
  const int block = h.block;
  const uint32_t bpr = (uint32_t)((h.p.nx + block - 1) / block);
  const int64_t nb = (int64_t)bpr * h.p.ny * h.p.nz;
  if (nb > 0x7fffffffLL) return hipErrorInvalidConfiguration;
  DirPtrs<T> P;
  for (int a = 0; a < 27; ++a) {
    P.src[a] = (const T*)src + (int64_t)a * h.stride;
    P.dst[a] = nullptr;
  }
  const dim3 grid((unsigned)nb), blk(block);
  switch (h.k.aa ? 2 : gather_kind(h)) {  // the AA layout keeps natural order: general slot rule
    case 0: hipLaunchKernelGGL((k_density<ST, 0>), grid, blk, 0, st, P, drho, h.k, bpr); break;
    case 1: hipLaunchKernelGGL((k_density<ST, 1>), grid, blk, 0, st, P, drho, h.k, bpr); break;
    default: hipLaunchKernelGGL((k_density<ST, 2>), grid, blk, 0, st, P, drho, h.k, bpr); break;
  }
  return hipGetLastError();
}

hipError_t launch_step(const lbm_handle& h, const void* src, void* dst, const float* force,
                       const float* grad_src, float* drho_out, hipStream_t st) {
  switch (h.p.storage) {
    case LBM_F32: return launch_step_t<0>(h, src, dst, force, grad_src, drho_out, st);
    case LBM_F16: return launch_step_t<1>(h, src, dst, force, grad_src, drho_out, st);
    default: return launch_step_t<2>(h, src, dst, force, grad_src, drho_out, st);
  }
}

template <int ST>
static hipError_t launch_step_aa_t(const lbm_handle& h, void* state, int odd, const float* force, hipStream_t st) {
  using T = typename Store<ST>::T;
  const int block = h.block;
  const uint32_t bpr = (uint32_t)((h.p.nx + block - 1) / block);
  const int64_t nb = (int64_t)bpr * h.p.ny * h.p.nz;
  if (nb > 0x7fffffffLL) return hipErrorInvalidConfiguration;
  DirPtrs<T> P;
  for (int a = 0; a < 27; ++a) {
    P.src[a] = (const T*)state + (int64_t)a * h.stride;
    P.dst[a] = (T*)state + (int64_t)a * h.stride;
  }
  const bool walls = h.k.bb_x || h.k.bb_y || h.k.bb_z;
  const dim3 grid((unsigned)nb), blk(block);
#define CLBM_AA(C, O, W, R) hipLaunchKernelGGL((k_step_aa<ST, C, O, W, R>), grid, blk, 0, st, P, force, h.k, bpr)
#define CLBM_AA_CORR(O, W, R)                 \
  switch (h.p.corr) {                         \
    case 0: CLBM_AA(0, O, W, R); break;       \
    case 1: CLBM_AA(1, O, W, R); break;       \
    default: CLBM_AA(2, O, W, R); break;      \
  }
#define CLBM_AA_RAW(O, W) \
  if (h.p.moments == LBM_RAW) { CLBM_AA_CORR(O, W, true) } else { CLBM_AA_CORR(O, W, false) }
  if (odd) {
    if (walls) { CLBM_AA_RAW(true, true) } else { CLBM_AA_RAW(true, false) }
  } else {
    if (walls) { CLBM_AA_RAW(false, true) } else { CLBM_AA_RAW(false, false) }
  }
#undef CLBM_AA_RAW
#undef CLBM_AA_CORR
#undef CLBM_AA
  return hipGetLastError();
}

hipError_t launch_step_aa(const lbm_handle& h, void* state, int odd, const float* force, hipStream_t st) {
  switch (h.p.storage) {
    case LBM_F32: return launch_step_aa_t<0>(h, state, odd, force, st);
    case LBM_F16: return launch_step_aa_t<1>(h, state, odd, force, st);
    default: return launch_step_aa_t<2>(h, state, odd, force, st);
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
    case LBM_F32: return launch_density_t<0>(h, src, drho, st);
    case LBM_F16: return launch_density_t<1>(h, src, drho, st);
    default: return launch_density_t<2>(h, src, drho, st);
  }
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
