// Kernels of the fused collide-and-stream step (two-buffer and in-place AA
// layouts) and their launchers, templated on the storage type.  Each storage
// type is instantiated in a translation unit of its own (lbm_step_<type>.hip)
// through StepKernels<ST>.
#pragma once

#include "lbm_internal.h"

namespace clbm {

// ------------------------------------------------------------------ step
// One thread per node, pull scheme: gather 27 slots of the source buffer,
// collide, write the node's 27 slots of the destination buffer (coalesced
// along x, non-temporal).  Without walls every source slot is
// (alpha, x - ebar_alpha) with periodic wrap, addressed as a per-direction
// base pointer plus a 32-bit node index shared by the three directions of
// one source row; with walls the slot rule of gather_slot applies (as 32-bit
// offsets from direction 0's array below 4 GiB, wall_slot32).  Periodic
// 16-bit grids with even nx run k_step_pair below instead, unless they use the
// full corrections.  With the full corrections (CORR 3) the density gradient comes from the
// density-deviation field grad_src, and drho_out (if not NULL) receives the
// node's own density deviation.
// HI: general rate of the moments of order >= 3 (k.omega_hi); false compiles
// the unit-rate collision.
// WALLS: 0 periodic (per-direction bases, 32-bit offsets), 1 walls with 32-bit
// offsets from direction 0's array (state below 4 GiB), 2 general (64-bit slots
// and field indices; walls, or periodic grids too large for kind 0).
// The directions with ebar_x = 0 are read with non-temporal loads (nt_dir).
template <int ST, int WALLS>
__device__ __forceinline__ void gather_node(const DirPtrs<typename Store<ST>::T>& P, int x, int y, int z,
                                            const Consts& k, float (&df)[27]) {
  constexpr int NT = 2;
  if constexpr (WALLS == 2) {
    gather_all<ST>(P.src[0], make_coord(x, y, z, k), k, df);
  } else {
    PeriodicRows pr;
    periodic_rows(x, y, z, k, pr);
    if constexpr (WALLS == 1) {
      const uint32_t node = ((uint32_t)z * (uint32_t)k.ny + (uint32_t)y) * (uint32_t)k.nx + (uint32_t)x;
      gather_walls32<ST, NT>(P.src[0], pr, node, wall_flags(x, y, z, k), k, df);
    } else {
      gather_periodic<ST, NT>(P.src, pr, k, df);
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

template <int ST, int CORR, int WALLS, bool RAW, bool HI>
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
    density_gradient_block<WALLS == 2>(grad_src, x, y, z, x < k.nx, k, lds, grx, gry, grz);
  }
  if (x >= k.nx) return;
  const uint32_t node = ((uint32_t)z * (uint32_t)k.ny + (uint32_t)y) * (uint32_t)k.nx + (uint32_t)x;
  float df[27];
  gather_node<ST, WALLS>(P, x, y, z, k, df);
  float fx = k.fx, fy = k.fy, fz = k.fz;
  if (force != nullptr) {
    fx = ld_field<WALLS == 2>(force, node);
    fy = ld_field<WALLS == 2>(force + k.n, node);
    fz = ld_field<WALLS == 2>(force + 2 * k.n, node);
  }
  float out[27];
  if constexpr (CORR == 3) {
    collide_node<CORR, RAW, HI>(df, fx, fy, fz, k, out, grx, gry, grz);
    if (drho_out != nullptr) drho_out[node] = low_moments(df).m000;
  } else {
    collide_node<CORR, RAW, HI>(df, fx, fy, fz, k, out);
  }
  if constexpr (ST == 0) conserve(df, fx, fy, fz, k, out);
  if constexpr (WALLS != 0) {
    if (k.moving) moving_wall_terms(x, y, z, k.rho0 + low_moments(df).m000, k, out);
  }
  const uint32_t so = store_offset(node);
#pragma unroll
  for (int a = 0; a < 27; ++a)
    st_off_nt(P.dst[a], so, Store<ST>::pack(ST == 0 ? out[a] : out[a] * k.sigma[wclass(a)]));
}

// ------------------------------------------------------------------ 16-bit step, two nodes per thread
// Periodic two-buffer step for FP16/BF16 storage with each thread owning the
// x-adjacent nodes 2t and 2t + 1: a 32-bit word of a direction array holds
// both nodes' values, so the gather is 27 aligned word loads (ebar_x = 0) or
// pairs of them (the x-shifted directions take one half from the neighbouring
// word) and the store 27 word stores; the two collisions run one after the
// other.  Measured on the bare access pattern at 512x512x256: 1.37 vs 1.45 ms
// for one node per thread with 2-byte accesses.  Results equal the one-node
// kernel's bit for bit (same gather values, same collision).
template <int ST, int A = 0>
__device__ __forceinline__ void gather_pair(const DirPtrs<typename Store<ST>::T>& P, const PeriodicRows& pr,
                                            uint32_t t, uint32_t tm, uint32_t tp, uint32_t (&w)[27]) {
  constexpr int ex = kEx[A];
  const uint32_t* base = reinterpret_cast<const uint32_t*>(P.src[A]);
  const uint32_t row = pr.row[kEy[A] + 1][kEz[A] + 1] / 2;      // word index of the source row
  if constexpr (ex == 0) {
    w[A] = ld_off_nt(base, row + t);                            // whole lines: non-temporal
  } else if constexpr (ex > 0) {                                // nodes 2t - 1, 2t
    const uint32_t own = ld_off(base, row + t), prev = ld_off(base, row + tm);
    w[A] = (prev >> 16) | (own << 16);
  } else {                                                      // nodes 2t + 1, 2t + 2
    const uint32_t own = ld_off(base, row + t), next = ld_off(base, row + tp);
    w[A] = (own >> 16) | (next << 16);
  }
  if constexpr (A + 1 < 27) gather_pair<ST, A + 1>(P, pr, t, tm, tp, w);
}

template <int ST, int CORR, bool RAW, bool HI>
__global__ __launch_bounds__(256) void k_step_pair(DirPtrs<typename Store<ST>::T> P, const float* __restrict__ force,
                                                   Consts k, uint32_t bpr) {
  static_assert(ST != 0, "two nodes per thread is the 16-bit path");
  const uint32_t lb = xcd_block(blockIdx.x, gridDim.x);
  const uint32_t bxi = lb % bpr, rowid = lb / bpr;
  const int y = (int)(rowid % (uint32_t)k.ny), z = (int)(rowid / (uint32_t)k.ny);
  const uint32_t tpr = (uint32_t)k.nx / 2;                      // words per row (nx even)
  const uint32_t t = bxi * blockDim.x + threadIdx.x;
  if (t >= tpr) return;
  const uint32_t tm = t == 0 ? tpr - 1 : t - 1, tp = t + 1 == tpr ? 0 : t + 1;
  PeriodicRows pr;
  periodic_rows((int)(2 * t), y, z, k, pr);
  uint32_t w[27];
  gather_pair<ST>(P, pr, t, tm, tp, w);
  const uint32_t node0 = pr.row[1][1] + 2 * t;
  PairWord<ST> o[27];
#pragma unroll
  for (int h = 0; h < 2; ++h) {
    float df[27];
#pragma unroll
    for (int a = 0; a < 27; ++a) df[a] = Store<ST>::from_bits(h ? w[a] >> 16 : w[a] & 0xffffu) * k.inv_sigma[wclass(a)];
    float fx = k.fx, fy = k.fy, fz = k.fz;
    if (force != nullptr) {
      fx = ld_off(force, node0 + h);
      fy = ld_off(force + k.n, node0 + h);
      fz = ld_off(force + 2 * k.n, node0 + h);
    }
    float out[27];
    collide_node<CORR, RAW, HI>(df, fx, fy, fz, k, out);
#pragma unroll
    for (int a = 0; a < 27; ++a) o[a].put(h, out[a] * k.sigma[wclass(a)]);
  }
  const uint32_t so = store_offset(pr.row[1][1] / 2 + t);
#pragma unroll
  for (int a = 0; a < 27; ++a) st_off_nt(reinterpret_cast<uint32_t*>(P.dst[a]), so, o[a].bits());
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
  // even steps read the node's own slots (no line shared between waves): all non-temporal;
  // odd steps as the two-buffer gather
  constexpr bool NT = !ODD || kEx[A] == 0;
  typename Store<ST>::T v;
  if constexpr (!ODD) {
    v = ld_pop<NT>(P.src[A], node);
  } else if constexpr (WALLS) {
    const uint32_t stride = (uint32_t)k.stride;
    const uint32_t idx = pulls_through_wall<A>(w) ? (uint32_t)A * stride + node
                                                  : (uint32_t)opp * stride + periodic_src<A>(pr);
    v = ld_pop<NT>(P.src[0], idx);
  } else {
    v = ld_pop<NT>(P.src[opp], periodic_src<A>(pr));
  }
  const float f = Store<ST>::load_val(v);
  df[A] = ST == 0 ? f : f * k.inv_sigma[wclass(A)];
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
  const typename Store<ST>::T v = Store<ST>::pack(ST == 0 ? out[A] : out[A] * k.sigma[wclass(A)]);
  if constexpr (!ODD) {
    st_off_nt(P.dst[opp], node, v);
  } else if constexpr (WALLS) {
    // x + ebar_A lies beyond a wall exactly when opp(A) pulls through one
    const uint32_t stride = (uint32_t)k.stride;
    const uint32_t idx = pulls_through_wall<opp>(w) ? (uint32_t)opp * stride + node
                                                    : (uint32_t)A * stride + periodic_src<opp>(pr);
    if constexpr (kEx[A] == 0) st_off_nt(P.dst[0], idx, v);
    else st_off(P.dst[0], idx, v);
  } else {
    // shifted by one node along x for 18 directions: plain stores, partial lines merge in L2;
    // the 9 with ebar_x = 0 write whole lines: non-temporal stores
    if constexpr (kEx[A] == 0) st_off_nt(P.dst[A], periodic_src<opp>(pr), v);
    else st_off(P.dst[A], periodic_src<opp>(pr), v);
  }
  if constexpr (A + 1 < 27) store_aa<ST, ODD, WALLS, A + 1>(P, pr, node, w, k, out);
}

template <int ST, int CORR, bool ODD, bool WALLS, bool RAW, bool HI>
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
  collide_node<CORR, RAW, HI>(df, fx, fy, fz, k, out);
  if constexpr (ST == 0) conserve(df, fx, fy, fz, k, out);
  if constexpr (WALLS) {
    if (k.moving) moving_wall_terms(x, y, z, k.rho0 + low_moments(df).m000, k, out);
  }
  // Store offsets defined next to the stores (store_offset), except in the FP32
  // odd step: there they cut the registers from 150 to 100, and the extra waves
  // let L2 evict the x-shifted partial lines before their second half arrives
  // (writes 113.9 instead of 109.3 B/LUP, 0.4% slower).
  if constexpr (ODD && ST == 0) store_aa<ST, ODD, WALLS>(P, pr, node, w, k, out);
  else if constexpr (ODD) store_aa<ST, ODD, WALLS>(P, store_rows(pr), store_offset(node), w, k, out);
  else store_aa<ST, ODD, WALLS>(P, pr, store_offset(node), w, k, out);
}

// 16-bit AA step with two x-adjacent nodes per thread (periodic grids, even nx;
// the pairing of k_step_pair).  Even steps read and write whole words of the
// node pair's own slots.  Odd steps gather like k_step_pair from the opposite
// directions' arrays; their x-shifted outputs land in words that two threads
// share, so those go out as 2-byte stores.
template <int ST, int A = 0>
__device__ __forceinline__ void gather_aa_pair(const DirPtrs<typename Store<ST>::T>& P, const PeriodicRows& pr,
                                               uint32_t t, uint32_t tm, uint32_t tp, bool odd, uint32_t (&w)[27]) {
  constexpr int ex = kEx[A];
  if (!odd) {
    w[A] = ld_off_nt(reinterpret_cast<const uint32_t*>(P.src[A]), pr.row[1][1] / 2 + t);
  } else {
    const uint32_t* base = reinterpret_cast<const uint32_t*>(P.src[opposite_of(A)]);
    const uint32_t row = pr.row[kEy[A] + 1][kEz[A] + 1] / 2;
    if constexpr (ex == 0) {
      w[A] = ld_off_nt(base, row + t);
    } else if constexpr (ex > 0) {
      const uint32_t own = ld_off(base, row + t), prev = ld_off(base, row + tm);
      w[A] = (prev >> 16) | (own << 16);
    } else {
      const uint32_t own = ld_off(base, row + t), next = ld_off(base, row + tp);
      w[A] = (own >> 16) | (next << 16);
    }
  }
  if constexpr (A + 1 < 27) gather_aa_pair<ST, A + 1>(P, pr, t, tm, tp, odd, w);
}

template <int ST, int A = 0>
__device__ __forceinline__ void store_aa_pair(const DirPtrs<typename Store<ST>::T>& P, const PeriodicRows& pr,
                                              uint32_t t, uint32_t tm, uint32_t tp, bool odd, const uint32_t (&o)[27]) {
  constexpr int ex = kEx[A];
  if (!odd) {
    st_off_nt(reinterpret_cast<uint32_t*>(P.dst[opposite_of(A)]), pr.row[1][1] / 2 + t, o[A]);
  } else {
    // f~_A of nodes 2t, 2t + 1 goes to (A, x + ebar_A)
    const uint32_t row = pr.row[1 - kEy[A]][1 - kEz[A]];       // row y + ey, z + ez (element index)
    if constexpr (ex == 0) {
      st_off_nt(reinterpret_cast<uint32_t*>(P.dst[A]), row / 2 + t, o[A]);
    } else {
      unsigned short* base = reinterpret_cast<unsigned short*>(P.dst[A]);
      const uint32_t lo = o[A] & 0xffffu, hi = o[A] >> 16;
      if constexpr (ex > 0) {                                    // positions 2t + 1, 2t + 2
        st_off(base, row + 2 * t + 1, (unsigned short)lo);
        st_off(base, row + 2 * tp, (unsigned short)hi);
      } else {                                                   // positions 2t - 1, 2t
        st_off(base, row + 2 * tm + 1, (unsigned short)lo);
        st_off(base, row + 2 * t, (unsigned short)hi);
      }
    }
  }
  if constexpr (A + 1 < 27) store_aa_pair<ST, A + 1>(P, pr, t, tm, tp, odd, o);
}

template <int ST, int CORR, bool ODD, bool RAW, bool HI>
__global__ __launch_bounds__(256) void k_step_aa_pair(DirPtrs<typename Store<ST>::T> P, const float* __restrict__ force,
                                                      Consts k, uint32_t bpr) {
  static_assert(ST != 0, "two nodes per thread is the 16-bit path");
  const uint32_t lb = xcd_block(blockIdx.x, gridDim.x);
  const uint32_t bxi = lb % bpr, rowid = lb / bpr;
  const int y = (int)(rowid % (uint32_t)k.ny), z = (int)(rowid / (uint32_t)k.ny);
  const uint32_t tpr = (uint32_t)k.nx / 2;
  const uint32_t t = bxi * blockDim.x + threadIdx.x;
  if (t >= tpr) return;
  const uint32_t tm = t == 0 ? tpr - 1 : t - 1, tp = t + 1 == tpr ? 0 : t + 1;
  PeriodicRows pr;
  periodic_rows((int)(2 * t), y, z, k, pr);
  uint32_t w[27];
  gather_aa_pair<ST>(P, pr, t, tm, tp, ODD, w);
  const uint32_t node0 = pr.row[1][1] + 2 * t;
  PairWord<ST> pw[27];
#pragma unroll
  for (int h = 0; h < 2; ++h) {
    float df[27];
#pragma unroll
    for (int a = 0; a < 27; ++a) df[a] = Store<ST>::from_bits(h ? w[a] >> 16 : w[a] & 0xffffu) * k.inv_sigma[wclass(a)];
    float fx = k.fx, fy = k.fy, fz = k.fz;
    if (force != nullptr) {
      fx = ld_off(force, node0 + h);
      fy = ld_off(force + k.n, node0 + h);
      fz = ld_off(force + 2 * k.n, node0 + h);
    }
    float out[27];
    collide_node<CORR, RAW, HI>(df, fx, fy, fz, k, out);
#pragma unroll
    for (int a = 0; a < 27; ++a) pw[a].put(h, out[a] * k.sigma[wclass(a)]);
  }
  uint32_t o[27];
#pragma unroll
  for (int a = 0; a < 27; ++a) o[a] = pw[a].bits();
  store_aa_pair<ST>(P, ODD ? store_rows(pr) : pr, store_offset(t), store_offset(tm), store_offset(tp), ODD, o);
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

// ------------------------------------------------------------------ launchers
// Gather path: 0 periodic, 32-bit byte offsets per direction array and into the
// force field (N floats, so N < 2^30 whatever the storage); 1 walls, 32-bit
// offsets across the whole state (below 4 GiB); 2 general, 64-bit slots and
// field indices (walls or periodic, any size).
static inline int gather_kind(const lbm_handle& h) {
  const bool walls = h.k.bb_x || h.k.bb_y || h.k.bb_z;
  if (!walls && (uint64_t)h.stride * 4u < (1ull << 32)) return 0;
  if (27ull * (uint64_t)h.stride * h.elem < (1ull << 32)) return 1;
  return 2;
}

template <int ST, bool HI>
static hipError_t launch_step_t(const lbm_handle& h, const void* src, void* dst, const float* force,
                                const float* grad_src, float* drho_out, hipStream_t st) {
  using T = typename Store<ST>::T;
  const int block = h.p.corr == LBM_CORR_FULL ? h.block : h.block_step;
  const uint32_t bpr = (uint32_t)((h.p.nx + block - 1) / block);
  const int64_t nb = (int64_t)bpr * h.p.ny * h.p.nz;
  if (nb > 0x7fffffffLL) return hipErrorInvalidConfiguration;
  DirPtrs<T> P;
  for (int a = 0; a < 27; ++a) {
    P.src[a] = (const T*)src + (int64_t)a * h.stride;
    P.dst[a] = (T*)dst + (int64_t)a * h.stride;
  }
  const int kind = gather_kind(h);
  if constexpr (ST != 0) {
    if (kind == 0 && h.pairs && h.p.corr != LBM_CORR_FULL && h.p.nx % 2 == 0) {
      constexpr int pblock = 128;                               // measured best of 64 / 128 / 256
      const uint32_t pbpr = (uint32_t)((h.p.nx / 2 + pblock - 1) / pblock);
      const int64_t pnb = (int64_t)pbpr * h.p.ny * h.p.nz;
      if (pnb > 0x7fffffffLL) return hipErrorInvalidConfiguration;
      const dim3 pgrid((unsigned)pnb), pblk(pblock);
#define CLBM_PAIR(C, R) hipLaunchKernelGGL((k_step_pair<ST, C, R, HI>), pgrid, pblk, 0, st, P, force, h.k, pbpr)
      const bool raw = h.p.moments == LBM_RAW;
      switch (h.p.corr) {
        case 0: if (raw) CLBM_PAIR(0, true); else CLBM_PAIR(0, false); break;
        case 1: if (raw) CLBM_PAIR(1, true); else CLBM_PAIR(1, false); break;
        default: if (raw) CLBM_PAIR(2, true); else CLBM_PAIR(2, false); break;
      }
#undef CLBM_PAIR
      return hipGetLastError();
    }
  }
  const dim3 grid((unsigned)nb), blk(block);
  const unsigned lds = h.p.corr == LBM_CORR_FULL ? 0u : (unsigned)h.step_lds;
#define CLBM_STEP(C, W, R) \
  hipLaunchKernelGGL((k_step<ST, C, W, R, HI>), grid, blk, lds, st, P, force, grad_src, drho_out, h.k, bpr)
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

template <int ST, bool HI>
static hipError_t launch_step_aa_t(const lbm_handle& h, void* state, int odd, const float* force, hipStream_t st) {
  using T = typename Store<ST>::T;
  const int block = h.block_step;
  const uint32_t bpr = (uint32_t)((h.p.nx + block - 1) / block);
  const int64_t nb = (int64_t)bpr * h.p.ny * h.p.nz;
  if (nb > 0x7fffffffLL) return hipErrorInvalidConfiguration;
  DirPtrs<T> P;
  for (int a = 0; a < 27; ++a) {
    P.src[a] = (const T*)state + (int64_t)a * h.stride;
    P.dst[a] = (T*)state + (int64_t)a * h.stride;
  }
  const bool walls = h.k.bb_x || h.k.bb_y || h.k.bb_z;
  if constexpr (ST != 0) {
    if (!walls && h.pairs && h.p.nx % 2 == 0) {
      constexpr int pblock = 128;
      const uint32_t pbpr = (uint32_t)((h.p.nx / 2 + pblock - 1) / pblock);
      const int64_t pnb = (int64_t)pbpr * h.p.ny * h.p.nz;
      if (pnb > 0x7fffffffLL) return hipErrorInvalidConfiguration;
      const dim3 pgrid((unsigned)pnb), pblk(pblock);
#define CLBM_AAP(C, O, R) hipLaunchKernelGGL((k_step_aa_pair<ST, C, O, R, HI>), pgrid, pblk, 0, st, P, force, h.k, pbpr)
#define CLBM_AAP_R(C, O) if (h.p.moments == LBM_RAW) CLBM_AAP(C, O, true); else CLBM_AAP(C, O, false)
      switch (h.p.corr) {
        case 0: if (odd) { CLBM_AAP_R(0, true); } else { CLBM_AAP_R(0, false); } break;
        case 1: if (odd) { CLBM_AAP_R(1, true); } else { CLBM_AAP_R(1, false); } break;
        default: if (odd) { CLBM_AAP_R(2, true); } else { CLBM_AAP_R(2, false); } break;
      }
#undef CLBM_AAP_R
#undef CLBM_AAP
      return hipGetLastError();
    }
  }
  const dim3 grid((unsigned)nb), blk(block);
#define CLBM_AA(C, O, W, R) \
  hipLaunchKernelGGL((k_step_aa<ST, C, O, W, R, HI>), grid, blk, (unsigned)h.step_lds, st, P, force, h.k, bpr)
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

template <int ST>
hipError_t StepKernels<ST>::step(const lbm_handle& h, const void* src, void* dst, const float* force,
                                 const float* grad_src, float* drho_out, hipStream_t st) {
  return h.k.hi ? launch_step_t<ST, true>(h, src, dst, force, grad_src, drho_out, st)
                : launch_step_t<ST, false>(h, src, dst, force, grad_src, drho_out, st);
}

template <int ST>
hipError_t StepKernels<ST>::step_aa(const lbm_handle& h, void* state, int odd, const float* force, hipStream_t st) {
  return h.k.hi ? launch_step_aa_t<ST, true>(h, state, odd, force, st)
                : launch_step_aa_t<ST, false>(h, state, odd, force, st);
}

template <int ST>
hipError_t StepKernels<ST>::density(const lbm_handle& h, const void* src, float* drho, hipStream_t st) {
  return launch_density_t<ST>(h, src, drho, st);
}

}  // namespace clbm
