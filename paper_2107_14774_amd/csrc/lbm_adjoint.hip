// Adjoint entry points: the reverse step (kernels in lbm_adjoint_step.h, one
// translation unit per storage type), the moving-wall terms, and the adjoint
// ends (observables, initialisation, natural order).
#include "lbm_adjoint_step.h"

namespace clbm {

// The adjoint arrays are in gathered-population order (lbm_adjoint_step.h):
// the element of slot (a, x) is the cotangent of what node x gathers as f_a.

// Transpose of the moving-wall terms of the forward store, -rho d_A with rho
// the sum of the node's gathered populations: the cotangent of every
// population the node gathered gains -sum_A lam_A d_A.  A separate pass after
// k_step_adjoint (it touches only nodes on a moving face and only their own
// elements, so no races), which keeps the main adjoint kernel's registers
// unchanged.
template <int A = 0>
__device__ __forceinline__ void add_to_own(float* __restrict__ dst, int x, int y, int z, const Consts& k, float v) {
  dst[slot_of<A>(x, y, z, k)] += v;
  if constexpr (A + 1 < 27) add_to_own<A + 1>(dst, x, y, z, k, v);
}

template <int A = 0>
__device__ __forceinline__ void store_own_all(float* __restrict__ dst, int x, int y, int z, const Consts& k,
                                              const float (&v)[27]) {
  dst[slot_of<A>(x, y, z, k)] = v[A];
  if constexpr (A + 1 < 27) store_own_all<A + 1>(dst, x, y, z, k, v);
}

__global__ __launch_bounds__(256) void k_moving_wall_adjoint(const float* __restrict__ adj_in, float* __restrict__ adj_out,
                                                             Consts k) {
  for (int64_t node = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; node < k.n;
       node += (int64_t)gridDim.x * blockDim.x) {
    const int x = (int)(node % k.nx);
    const int64_t t = node / k.nx;
    const int y = (int)(t % k.ny), z = (int)(t / k.ny);
    const bool on_moving = (k.bb_x && (((k.moving & 1) && x == 0) || ((k.moving & 2) && x == k.nx - 1))) ||
                           (k.bb_y && (((k.moving & 4) && y == 0) || ((k.moving & 8) && y == k.ny - 1))) ||
                           (k.bb_z && (((k.moving & 16) && z == 0) || ((k.moving & 32) && z == k.nz - 1)));
    if (!on_moving) continue;
    float lam[27];
    load_next_all(adj_in, make_coord(x, y, z, k), k, lam);   // lambda(t+1) of the node's own slots
    const float c = moving_wall_vjp(x, y, z, k, lam);
    add_to_own(adj_out, x, y, z, k, -c);
  }
}

// Transpose of the full corrections' density gradient (density_gradient_block:
// grad rho(x) = sum_a c_a rho(nb(x, a)), nb the neighbour x + ebar_a with each
// axis clamped at a wall), followed by d rho / d f = 1: every population node y
// gathered gains g_rho(y) = sum_a sum_{x : nb(x, a) = y} c_a . gg(x), gg the
// cotangent of the gradient that k_step_adjoint wrote.  Per axis the sources of
// y are y - e (periodic: wrapped), plus y itself at a wall the shift points out of.
//
// The stencil's coefficients factorise like the forward's (density_gradient_block):
//   c_a = (0.5 ex Wy Wz, 0.5 ic_y ey Wx Wz, 0.5 ic_z ez Wx Wy),
// so each thread reduces the transverse (y, z) sources of its own column X into
//   A(X) = sum Wy Wz ggx,  B(X) = sum ey Wz ggy,  C(X) = sum Wy ez ggz
// (the sources of the block's row), and the x shift combines neighbouring
// columns through LDS: g_rho(x) = sum_ex [0.5 ex A + 0.5 (ic_y B + ic_z C) Wx(ex)](X)
// over the x sources X of each ex.
//
// Grouped by source row, the transverse sums read the rows at offsets -1, 0, +1 in y and in z
// with per-axis weights (the sum of W(e), resp. of e, over the shifts e whose source is that row):
// nine rows of each component, all known to the whole block (one row per block).
struct AxisWeights {
  int row[3];       // source row at offset o = -1, 0, +1 (wrapped, or clamped where its weight is 0)
  float w[3], e[3];
};

__device__ __forceinline__ AxisWeights axis_weights(int v, int n, bool wall, float wc, float ws) {
  AxisWeights a;
#pragma unroll
  for (int i = 0; i < 3; ++i) {
    a.w[i] = 0.0f;
    a.e[i] = 0.0f;
    int r = v + i - 1;
    if (wall) r = r < 0 ? 0 : (r >= n ? n - 1 : r);
    else r = r < 0 ? r + n : (r >= n ? r - n : r);
    a.row[i] = r;
  }
#pragma unroll
  for (int e = -1; e <= 1; ++e) {
    const float w = e == 0 ? wc : ws;
    const int p = v - e;  // the source the shift e reads from (offset -e)
    if (!wall || (p >= 0 && p < n)) { a.w[1 - e] += w; a.e[1 - e] += (float)e; }
    if (wall && e != 0 && ((e < 0 && v == 0) || (e > 0 && v == n - 1))) { a.w[1] += w; a.e[1] += (float)e; }
  }
  return a;
}

struct TransverseWeights {
  int64_t base[3][3];            // element index of source row (z offset, y offset), x = 0
  float a[3][3], b[3][3], c[3][3];
};

__device__ __forceinline__ TransverseWeights transverse_weights(int y, int z, const Consts& k) {
  const AxisWeights ay = axis_weights(y, k.ny, k.bb_y, k.w0c[1], k.w0s[1]);
  const AxisWeights az = axis_weights(z, k.nz, k.bb_z, k.w0c[2], k.w0s[2]);
  TransverseWeights t;
#pragma unroll
  for (int iz = 0; iz < 3; ++iz)
#pragma unroll
    for (int iy = 0; iy < 3; ++iy) {
      t.base[iz][iy] = ((int64_t)az.row[iz] * k.ny + ay.row[iy]) * k.nx;
      t.a[iz][iy] = az.w[iz] * ay.w[iy];
      t.b[iz][iy] = az.w[iz] * ay.e[iy];
      t.c[iz][iy] = az.e[iz] * ay.w[iy];
    }
  return t;
}

__device__ __forceinline__ void transverse_column(const float* __restrict__ gg, int X, const TransverseWeights& t,
                                                  const Consts& k, float& A, float& B, float& C) {
  A = 0.0f; B = 0.0f; C = 0.0f;
#pragma unroll
  for (int iz = 0; iz < 3; ++iz)
#pragma unroll
    for (int iy = 0; iy < 3; ++iy) {
      // every row index is valid (clamped where the weight is 0), so all 27 loads issue together;
      // uniform row pointers and one 32-bit x offset (SGPR base + VGPR offset addressing)
      const float* r0 = gg + t.base[iz][iy];
      const float g0 = ld_off(r0, (uint32_t)X), g1 = ld_off(r0 + k.n, (uint32_t)X), g2 = ld_off(r0 + 2 * k.n, (uint32_t)X);
      A += t.a[iz][iy] * g0;
      B += t.b[iz][iy] * g1;
      C += t.c[iz][iy] * g2;
    }
}

// v added to the node's 27 own elements (row start, chunk, x offset)
template <int A = 0>
__device__ __forceinline__ void add_own_row(float* __restrict__ row, uint32_t xo, float v) {
  float* p = row + chunk_of(A) * kB + xo;
  *p += v;
  if constexpr (A + 1 < 27) add_own_row<A + 1>(row, xo, v);
}

// One block per row segment (like the step); every thread of the block calls the barrier.
// FIELD: write the node's sum to out[node] (natural node order) instead of adding it to the node's
// 27 own adjoint elements.
template <bool FIELD>
__global__ __launch_bounds__(256) void k_density_vjp(const float* __restrict__ gg, float* __restrict__ out, Consts k,
                                                     uint32_t bpr) {
  const uint32_t lb = xcd_block(blockIdx.x, gridDim.x);
  const uint32_t bxi = lb % bpr, rowid = lb / bpr;
  int y, z;
  tiled_row(rowid, (uint32_t)k.ytile, k, y, z);  // y-tiles, as the gradient's forward pass
  const int x = (int)(bxi * blockDim.x + threadIdx.x);
  const int t = (int)threadIdx.x;
  const bool active = x < k.nx;
  // lds[c][t + 1]: column x of the block; [0] and [blockDim + 1]: the columns left and right of it
  __shared__ float lds[3][258];
  const TransverseWeights tw = transverse_weights(y, z, k);
  if (active) {
    float A, B, C;
    transverse_column(gg, x, tw, k, A, B, C);
    lds[0][t + 1] = A; lds[1][t + 1] = B; lds[2][t + 1] = C;
    if (t == 0 && x > 0) {
      transverse_column(gg, x - 1, tw, k, A, B, C);
      lds[0][0] = A; lds[1][0] = B; lds[2][0] = C;
    }
    if ((t == (int)blockDim.x - 1 || x == k.nx - 1) && x < k.nx - 1) {
      transverse_column(gg, x + 1, tw, k, A, B, C);
      lds[0][t + 2] = A; lds[1][t + 2] = B; lds[2][t + 2] = C;
    }
  }
  __syncthreads();
  if (!active) return;
  // the row's ends: a periodic x wraps to the other end of the row, which another block holds
  float Am, Bm, Cm, Ap, Bp, Cp;
  if (x > 0) { Am = lds[0][t]; Bm = lds[1][t]; Cm = lds[2][t]; }
  else transverse_column(gg, k.nx - 1, tw, k, Am, Bm, Cm);
  if (x < k.nx - 1) { Ap = lds[0][t + 2]; Bp = lds[1][t + 2]; Cp = lds[2][t + 2]; }
  else transverse_column(gg, 0, tw, k, Ap, Bp, Cp);
  const float A0 = lds[0][t + 1], B0 = lds[1][t + 1], C0 = lds[2][t + 1];
  const float hy = 0.5f * k.ic[1], hz = 0.5f * k.ic[2];
  const float wc = k.w0c[0], ws = k.w0s[0];
  // ex = 0: the column itself
  float g = wc * (hy * B0 + hz * C0);
  // ex = +1: source x - 1 (at an x wall, x = 0 has none; x = nx - 1 also itself)
  // ex = -1: source x + 1 (at an x wall, x = nx - 1 has none; x = 0 also itself)
  const bool wx = k.bb_x;
  const bool has_m = !(wx && x == 0), has_p = !(wx && x == k.nx - 1);
  if (has_m) g += 0.5f * Am + ws * (hy * Bm + hz * Cm);
  if (has_p) g += -0.5f * Ap + ws * (hy * Bp + hz * Cp);
  if (wx && x == k.nx - 1) g += 0.5f * A0 + ws * (hy * B0 + hz * C0);
  if (wx && x == 0) g += -0.5f * A0 + ws * (hy * B0 + hz * C0);
  if constexpr (FIELD) st_off(out + ((int64_t)z * k.ny + y) * k.nx, (uint32_t)x, g);
  else add_own_row(out + row_start(y, z, k), xoff((uint32_t)x), g);
}

// ------------------------------------------------------------------ observables adjoint
template <int ST>
__global__ __launch_bounds__(256) void k_moments_adjoint(const typename Store<ST>::T* __restrict__ state,
                                                         const float* __restrict__ force, const float* __restrict__ g_rho,
                                                         const float* __restrict__ g_u, float* __restrict__ adj,
                                                         float* __restrict__ grad_force, Consts k) {
  for (int64_t node = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; node < k.n;
       node += (int64_t)gridDim.x * blockDim.x) {
    const int x = (int)(node % k.nx);
    const int64_t t = node / k.nx;
    const NodeCoord c = make_coord(x, (int)(t % k.ny), (int)(t / k.ny), k);
    float df[27];
    gather_all<ST>(state, c, k, df);
    const LowMoments M = low_moments(df);
    float fx = k.fx, fy = k.fy, fz = k.fz;
    if (force != nullptr) {
      fx = force[node];
      fy = force[k.n + node];
      fz = force[2 * k.n + node];
    }
    const float rho = k.rho0 + M.m000;
    const float irho = 1.0f / rho;
    const float ux = (M.m100 + 0.5f * fx) * irho, uy = (k.r * M.m010 + 0.5f * fy) * irho;
    const float uz = (k.s * M.m001 + 0.5f * fz) * irho;
    const float gr = g_rho ? g_rho[node] : 0.0f;
    const float gx = g_u ? g_u[node] : 0.0f, gy = g_u ? g_u[k.n + node] : 0.0f, gz = g_u ? g_u[2 * k.n + node] : 0.0f;
    const float brho = gr - (gx * ux + gy * uy + gz * uz) * irho;
    const float bj[3] = {gx * irho, k.r * gy * irho, k.s * gz * irho};
    float mu[27];
#pragma unroll
    for (int a = 0; a < 27; ++a) {
      float v = brho;
      if (kEx[a] != 0) v += kEx[a] * bj[0];
      if (kEy[a] != 0) v += kEy[a] * bj[1];
      if (kEz[a] != 0) v += kEz[a] * bj[2];
      mu[a] = v;
    }
    store_own_all(adj, c.x, c.y, c.z, k, mu);
    if (grad_force != nullptr) {
      grad_force[node] += 0.5f * gx * irho;
      grad_force[k.n + node] += 0.5f * gy * irho;
      grad_force[2 * k.n + node] += 0.5f * gz * irho;
    }
  }
}

// ------------------------------------------------------------------ init adjoint (FP64)
template <int A = 0>
__device__ __forceinline__ void own_adj(const float* __restrict__ adj, const NodeCoord& c, const Consts& k,
                                        double (&l)[27]) {
  l[A] = (double)adj[slot_of<A>(c.x, c.y, c.z, k)];
  if constexpr (A + 1 < 27) own_adj<A + 1>(adj, c, k, l);
}

__global__ __launch_bounds__(256) void k_init_adjoint(const float* __restrict__ adj, const double* __restrict__ rho,
                                                      const double* __restrict__ u, double* __restrict__ g_rho,
                                                      double* __restrict__ g_u, Consts k, ConstsD kd) {
  for (int64_t node = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; node < k.n;
       node += (int64_t)gridDim.x * blockDim.x) {
    const int x = (int)(node % k.nx);
    const int64_t t = node / k.nx;
    const NodeCoord c = make_coord(x, (int)(t % k.ny), (int)(t / k.ny), k);
    double l[27];
    own_adj(adj, c, k, l);
    const double rn = rho ? rho[node] : kd.rho0;
    const double uu[3] = {u ? u[node] : 0.0, u ? u[k.n + node] : 0.0, u ? u[2 * k.n + node] : 0.0};
    double E[3][3], A1[3][3];
    for (int d = 0; d < 3; ++d) {
      const double q = uu[d] * uu[d] * kd.ic2[d], h = uu[d] * kd.ic[d];
      E[d][0] = kd.w0s[d] + 0.5 * (q - h);
      E[d][1] = kd.w0c[d] - q;
      E[d][2] = kd.w0s[d] + 0.5 * (q + h);
      const double uic2 = uu[d] * kd.ic2[d], hic = 0.5 * kd.ic[d];
      A1[d][0] = uic2 - hic;
      A1[d][1] = -2.0 * uic2;
      A1[d][2] = uic2 + hic;
    }
    // f_eq = rho E_x (x) E_y (x) E_z: d/drho = E E E, d/du_d = rho (E with E_d replaced by A1_d)
    double gr = 0.0, gx = 0.0, gy = 0.0, gz = 0.0;
#pragma unroll
    for (int i = 0; i < 3; ++i)
#pragma unroll
      for (int j = 0; j < 3; ++j) {
        double lE = 0.0, lA = 0.0;
#pragma unroll
        for (int m = 0; m < 3; ++m) {
          const double lv = l[dir_of(i, j, m)];
          lE += lv * E[2][m];
          lA += lv * A1[2][m];
        }
        gr += lE * E[0][i] * E[1][j];
        gx += lE * A1[0][i] * E[1][j];
        gy += lE * E[0][i] * A1[1][j];
        gz += lA * E[0][i] * E[1][j];
      }
    if (g_rho) g_rho[node] = gr;
    if (g_u) {
      g_u[node] = rn * gx;
      g_u[k.n + node] = rn * gy;
      g_u[2 * k.n + node] = rn * gz;
    }
  }
}

// ------------------------------------------------------------------ slots <-> natural order
template <int A = 0>
__device__ __forceinline__ void slots_to_nat(const float* __restrict__ s, const NodeCoord& c, int64_t node,
                                             double* __restrict__ nat, const Consts& k) {
  nat[A * k.n + node] = (double)s[slot_of<A>(c.x, c.y, c.z, k)];
  if constexpr (A + 1 < 27) slots_to_nat<A + 1>(s, c, node, nat, k);
}

template <int A = 0>
__device__ __forceinline__ void nat_to_slots(const double* __restrict__ nat, const NodeCoord& c, int64_t node,
                                             float* __restrict__ s, const Consts& k) {
  s[slot_of<A>(c.x, c.y, c.z, k)] = (float)nat[A * k.n + node];
  if constexpr (A + 1 < 27) nat_to_slots<A + 1>(nat, c, node, s, k);
}

__global__ __launch_bounds__(256) void k_adjoint_natural(const float* __restrict__ slots, double* __restrict__ natural,
                                                         int to_natural, const double* __restrict__ natural_in,
                                                         float* __restrict__ slots_out, Consts k) {
  for (int64_t node = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; node < k.n;
       node += (int64_t)gridDim.x * blockDim.x) {
    const int x = (int)(node % k.nx);
    const int64_t t = node / k.nx;
    const NodeCoord c = make_coord(x, (int)(t % k.ny), (int)(t / k.ny), k);
    if (to_natural) slots_to_nat(slots, c, node, natural, k);
    else nat_to_slots(natural_in, c, node, slots_out, k);
  }
}

// ------------------------------------------------------------------ launchers
static int grid_cap(int64_t n, int cap) {
  int64_t g = (n + 255) / 256;
  return (int)(g < 1 ? 1 : (g > cap ? cap : g));
}

// The stencil's transpose of a gradient cotangent: added to every own element of an adjoint array
// (field = false), or written as one value per node into out[n] (field = true).
static hipError_t launch_density_vjp(const lbm_handle& h, const float* grad, float* out, bool field, hipStream_t st) {
  const int block = h.block;
  const uint32_t bpr = (uint32_t)((h.p.nx + block - 1) / block);
  const int64_t nb = (int64_t)bpr * h.p.ny * h.p.nz;
  if (nb > 0x7fffffffLL) return hipErrorInvalidConfiguration;
  if (field) hipLaunchKernelGGL(k_density_vjp<true>, dim3((unsigned)nb), dim3(block), 0, st, grad, out, h.k, bpr);
  else hipLaunchKernelGGL(k_density_vjp<false>, dim3((unsigned)nb), dim3(block), 0, st, grad, out, h.k, bpr);
  return hipGetLastError();
}

hipError_t launch_density_adjoint(const lbm_handle& h, const float* grad, float* adj, hipStream_t st) {
  return launch_density_vjp(h, grad, adj, false, st);
}

hipError_t launch_step_adjoint(const lbm_handle& h, const void* state, const float* adj_in, float* adj_out,
                               const float* force, float* grad_force, double* grad_force_uniform, float* drho,
                               float* grad_rho, bool exact, bool drho_given, const float* pending,
                               hipStream_t st) {
  const bool full = h.p.corr == LBM_CORR_FULL;
  hipError_t e = hipSuccess;
  // the density field the step's gradient came from
  if (full && exact && !drho_given) e = launch_density(h, state, drho, st);
  if (e != hipSuccess) return e;
  // lagged: the next step took its gradient from this state's density, so the stencil's transpose of
  // its cotangent (pending) belongs to every population of this state.  It goes, one value per node,
  // into the first component of grad_rho, which the adjoint kernel reads before it writes the element
  // and adds to the node's own outputs (instead of a pass over the 27 outputs afterwards).
  const bool pend = full && !exact && pending != nullptr;
  if (pend) e = launch_density_vjp(h, pending, grad_rho, true, st);
  if (e != hipSuccess) return e;
  switch (h.p.storage) {
    case LBM_F32: e = AdjointKernels<0>::step(h, state, adj_in, adj_out, force, grad_force, grad_force_uniform, drho,
                                              grad_rho, pend, st); break;
    case LBM_F16: e = AdjointKernels<1>::step(h, state, adj_in, adj_out, force, grad_force, grad_force_uniform, drho,
                                              grad_rho, pend, st); break;
    default: e = AdjointKernels<2>::step(h, state, adj_in, adj_out, force, grad_force, grad_force_uniform, drho,
                                         grad_rho, pend, st); break;
  }
  if (e != hipSuccess) return e;
  if (h.k.moving) {
    int64_t g = (h.n + 255) / 256;
    if (g > 65536) g = 65536;
    hipLaunchKernelGGL(k_moving_wall_adjoint, (unsigned)g, 256, 0, st, adj_in, adj_out, h.k);
    e = hipGetLastError();
    if (e != hipSuccess) return e;
  }
  // exact: this step's gradient came from this state
  if (full && exact) e = launch_density_adjoint(h, grad_rho, adj_out, st);
  return e;
}

hipError_t launch_moments_adjoint(const lbm_handle& h, const void* state, const float* force, const float* g_rho,
                                  const float* g_u, float* adj, float* grad_force, hipStream_t st) {
  const int g = grid_cap(h.n, 65536);
  switch (h.p.storage) {
    case LBM_F32:
      hipLaunchKernelGGL(k_moments_adjoint<0>, g, 256, 0, st, (const float*)state, force, g_rho, g_u, adj, grad_force, h.k);
      break;
    case LBM_F16:
      hipLaunchKernelGGL(k_moments_adjoint<1>, g, 256, 0, st, (const Store<1>::T*)state, force, g_rho, g_u, adj,
                         grad_force, h.k);
      break;
    default:
      hipLaunchKernelGGL(k_moments_adjoint<2>, g, 256, 0, st, (const Store<2>::T*)state, force, g_rho, g_u, adj,
                         grad_force, h.k);
      break;
  }
  return hipGetLastError();
}

hipError_t launch_init_adjoint(const lbm_handle& h, const float* adj, const double* rho, const double* u, double* g_rho,
                               double* g_u, hipStream_t st) {
  hipLaunchKernelGGL(k_init_adjoint, grid_cap(h.n, 65536), 256, 0, st, adj, rho, u, g_rho, g_u, h.k, h.kd);
  return hipGetLastError();
}

hipError_t launch_adjoint_natural(const lbm_handle& h, const float* slots, double* natural, int to_natural,
                                  const double* natural_in, float* slots_out, hipStream_t st) {
  hipLaunchKernelGGL(k_adjoint_natural, grid_cap(h.n, 65536), 256, 0, st, slots, natural, to_natural, natural_in,
                     slots_out, h.k);
  return hipGetLastError();
}

}  // namespace clbm
