// Kernels of the fused collide-and-stream step (two-buffer and in-place AA
// layouts) and their launchers, templated on the storage type.  Each storage
// type is instantiated in a translation unit of its own (lbm_step_<type>.hip)
// through StepKernels<ST>.
#pragma once

#include "lbm_internal.h"

// Loads of the gathers: 2 = non-temporal for the directions with ebar_x = 0,
// plain for the x-shifted ones (nt_dir); 1 = non-temporal for all 27.
#ifndef LBM_GATHER_NT
#define LBM_GATHER_NT 2
#endif

namespace clbm {

// ------------------------------------------------------------------ step
// One thread per node, pull scheme: gather 27 slots of the source buffer,
// collide, write the node's 27 slots of the destination buffer (coalesced
// along x, non-temporal).  Without walls every source slot is
// (alpha, x - ebar_alpha) with periodic wrap, addressed as the scalar start of
// the source row plus a per-lane offset (any state size); with walls the slot
// rule of gather_slot applies, as 32-bit offsets from the start of the state
// below 4 GiB (wall_slot32) and as 64-bit slots above.  Periodic 16-bit grids
// with even nx run k_step_pair (or, with the full corrections,
// k_step_full_pair) below instead.  With the full corrections (CORR 3) the density gradient comes
// from the density-deviation field grad_src, and drho_out (if not NULL)
// receives the node's own density deviation.
// HI: general rate of the moments of order >= 3 (k.omega_hi); false compiles
// the unit-rate collision.
// WALLS: 0 periodic (row addresses), 1 walls with 32-bit offsets (state below
// 4 GiB), 2 general (64-bit slots).
template <int ST, int WALLS>
__device__ __forceinline__ void gather_node(const typename Store<ST>::T* __restrict__ src, const Upstream& u, int x,
                                            int y, int z, const Consts& k, float (&df)[27]) {
  constexpr int NT = LBM_GATHER_NT;
  if constexpr (WALLS == 2) {
    gather_all<ST>(src, make_coord(x, y, z, k), k, df);
  } else if constexpr (WALLS == 1) {
    gather_walls32<ST, NT>(src, u, wall_flags(x, y, z, k), k, df);
  } else {
    gather_periodic<ST, NT>(pull_groups(src, u), u, k, df);
  }
}

// The node's 27 post-collision values into its own slots of dst (coalesced,
// non-temporal), in issue order.
// r16: the node's random bits of the stochastic rounding (BF16-SR storage only).
template <int ST, int I = 0>
__device__ __forceinline__ void store_own(const GroupBases<typename Store<ST>::T>& d, uint32_t so,
                                          const float (&out)[27], const Consts& k, uint32_t r16) {
  constexpr int a = issue_dir(I);
  st_off_nt(chunk_ptr<a>(d), so, pack_rounded<ST>(encode_scale<ST>(out[a], wclass(a), k), r16));
  if constexpr (I + 1 < 27) store_own<ST, I + 1>(d, so, out, k, r16);
}

// Random bits of the stochastic rounding of node `node` in this step (0 unless BF16-SR).
template <int ST>
__device__ __forceinline__ uint32_t node_sr_bits(uint32_t node, const Consts& k) {
  if constexpr (ST == 3) return sr_bits(node, k.seq_hash);
  else return 0u;
}

// Body force of a node: the uniform one, or the field's value through the
// scalar start of the node's row (natural order, any field size).
__device__ __forceinline__ void node_force(const float* __restrict__ force, int64_t nrow, uint32_t x, const Consts& k,
                                           float& fx, float& fy, float& fz) {
  fx = k.fx; fy = k.fy; fz = k.fz;
  if (force != nullptr) {
    const float* f = force + nrow;
    fx = ld_off(f, x);
    fy = ld_off(f + k.n, x);
    fz = ld_off(f + 2 * k.n, x);
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
__global__ __launch_bounds__(256, step_waves(ST, CORR)) void k_step(const typename Store<ST>::T* __restrict__ src,
                                                                    typename Store<ST>::T* __restrict__ dst,
                                                                    const float* __restrict__ force,
                                                                    const float* __restrict__ grad_src,
                                                                    float* __restrict__ drho_out, Consts k,
                                                                    uint32_t bpr) {
  const uint32_t lb = xcd_block(blockIdx.x, gridDim.x);
  const uint32_t bxi = lb % bpr, rowid = lb / bpr;
  // the full-correction step walks y-tiles of k.ytile rows, z-major inside a tile: the density
  // rows of z - 1 and z + 1 are then read a few rows apart (an L2 hit) instead of a plane apart
  int y, z;
  tiled_row(rowid, (uint32_t)(CORR == 3 ? k.ytile : 1), k, y, z);
  const int x = (int)(bxi * blockDim.x + threadIdx.x);
  // the density gradient first (block-wide, with a barrier), while no population is live
  float grx = 0.0f, gry = 0.0f, grz = 0.0f;
  if constexpr (CORR == 3) {
    __shared__ float lds[3][258];
    density_gradient_block(grad_src, x, y, z, x < k.nx, k, lds, grx, gry, grz);
  }
  if (x >= k.nx) return;
  Upstream u;
  upstream(x, y, z, k, u);
  float df[27];
  gather_node<ST, WALLS>(src, u, x, y, z, k, df);
  const int64_t nrow = ((int64_t)z * k.ny + y) * k.nx;
  float fx, fy, fz;
  node_force(force, nrow, (uint32_t)x, k, fx, fy, fz);
  float out[27];
  if constexpr (CORR == 3) {
    collide_fenced<CORR, RAW, HI, ST == 0 || HI>(df, fx, fy, fz, k, out, grx, gry, grz);
    if (drho_out != nullptr) st_off(drho_out + nrow, (uint32_t)x, low_moments(df).m000);
  } else {
    collide_fenced<CORR, RAW, HI, ST == 0 || HI>(df, fx, fy, fz, k, out);
  }
  if constexpr (ST == 0) conserve(df, fx, fy, fz, k, out);
  if constexpr (WALLS != 0) {
    if (k.moving) moving_wall_terms(x, y, z, k.rho0 + low_moments(df).m000, k, out);
  }
  store_own<ST>(own_groups(dst, u), store_offset(u.xo[1]), out, k, node_sr_bits<ST>((uint32_t)nrow + x, k));
}

// ------------------------------------------------------------------ 16-bit step, two nodes per thread
// Periodic two-buffer step for FP16/BF16 storage with each thread owning the
// x-adjacent nodes 2t and 2t + 1: a 32-bit word of a chunk holds both nodes'
// values, so the gather is 27 aligned word loads (ebar_x = 0) or pairs of them
// (the x-shifted directions take one half from the neighbouring word) and the
// store 27 word stores; the two collisions run one after the other.  Results
// equal the one-node kernel's bit for bit (same gather values, same collision).

// Word offset of word t (nodes 2t, 2t + 1) within a row: xoff(2t) / 2.
__device__ __forceinline__ uint32_t xoffw(uint32_t t) {
  return (t / (kB / 2)) * (27u * kB / 2) + t % (kB / 2);
}

// Word offsets of the words t + 1, t, t - 1 (wrapped), indexed like Upstream::xo.
struct PairWords {
  uint32_t xw[3];
};

__device__ __forceinline__ PairWords pair_words(uint32_t t, uint32_t tm, uint32_t tp) {
  PairWords p;
  p.xw[0] = xoffw(tp);
  p.xw[1] = xoffw(t);
  p.xw[2] = xoffw(tm);
  return p;
}

// Words of a 16-bit chunk (chunks start on even elements).
template <typename T>
__device__ __forceinline__ const global_t<uint32_t>* words(const global_t<T>* chunk) {
  return reinterpret_cast<const global_t<uint32_t>*>(chunk);
}
template <typename T>
__device__ __forceinline__ global_t<uint32_t>* words(global_t<T>* chunk) {
  return reinterpret_cast<global_t<uint32_t>*>(chunk);
}

// The two values f_A of nodes 2t, 2t + 1 from the chunk `chunk` holding the
// slots of the nodes upstream of A (its own slots in the pull step, the
// opposite direction's in the AA odd step): one word (ebar_x = 0) or the
// halves of two (ebar_x != 0).
template <int A, typename T>
__device__ __forceinline__ uint32_t pair_gather_word(const global_t<T>* chunk, const PairWords& p) {
  constexpr int ex = kEx[A];
  const global_t<uint32_t>* base = words(chunk);
  if constexpr (ex == 0) {
    return ld_off_nt(base, p.xw[1]);                            // whole lines: non-temporal
  } else if constexpr (ex > 0) {                                // nodes 2t - 1, 2t
    const uint32_t own = ld_pop<LBM_GATHER_NT == 1>(base, p.xw[1]), prev = ld_pop<LBM_GATHER_NT == 1>(base, p.xw[2]);
    return (prev >> 16) | (own << 16);
  } else {                                                      // nodes 2t + 1, 2t + 2
    const uint32_t own = ld_pop<LBM_GATHER_NT == 1>(base, p.xw[1]), next = ld_pop<LBM_GATHER_NT == 1>(base, p.xw[0]);
    return (own >> 16) | (next << 16);
  }
}

template <int ST, int I = 0>
__device__ __forceinline__ void gather_pair(const GroupBases<const typename Store<ST>::T>& b, const PairWords& p,
                                            uint32_t (&w)[27]) {
  constexpr int A = issue_dir(I);
  w[A] = pair_gather_word<A>(chunk_ptr<A>(b), p);
  if constexpr (I + 1 < 27) gather_pair<ST, I + 1>(b, p, w);
}

template <int ST, int I = 0>
__device__ __forceinline__ void store_pair_own(const GroupBases<typename Store<ST>::T>& d, uint32_t so,
                                               const uint32_t (&o)[27]) {
  constexpr int a = issue_dir(I);
  st_off_nt(words(chunk_ptr<a>(d)), so, o[a]);
  if constexpr (I + 1 < 27) store_pair_own<ST, I + 1>(d, so, o);
}

// Decode, collide and encode the two nodes of a pair (shared by the two-buffer
// and AA pair steps).
template <int ST, int CORR, bool RAW, bool HI>
__device__ __forceinline__ void collide_pair(const uint32_t (&w)[27], const float* __restrict__ force, int64_t nrow,
                                             uint32_t x0, const Consts& k, uint32_t (&o)[27]) {
  PairWord<ST> pw[27];
#pragma unroll
  for (int h = 0; h < 2; ++h) {
    float df[27];
#pragma unroll
    for (int a = 0; a < 27; ++a) df[a] = decode_scale<ST>(word_half<ST>(w[a], h), wclass(a), k);
    float fx, fy, fz;
    node_force(force, nrow, x0 + h, k, fx, fy, fz);
    float out[27];
    collide_fenced<CORR, RAW, HI, ST == 0 || HI>(df, fx, fy, fz, k, out);
    if constexpr (ST == 3) {
      const uint32_t r16 = sr_bits((uint32_t)nrow + x0 + h, k.seq_hash);
#pragma unroll
      for (int a = 0; a < 27; ++a) pw[a].put(h, out[a], r16);
    } else {
#pragma unroll
      for (int a = 0; a < 27; ++a) pw[a].put(h, encode_scale<ST>(out[a], wclass(a), k));
    }
  }
#pragma unroll
  for (int a = 0; a < 27; ++a) o[a] = pw[a].bits();
}

template <int ST, int CORR, bool RAW, bool HI>
__global__ __launch_bounds__(256) void k_step_pair(const typename Store<ST>::T* __restrict__ src,
                                                   typename Store<ST>::T* __restrict__ dst,
                                                   const float* __restrict__ force, Consts k, uint32_t bpr) {
  static_assert(ST != 0, "two nodes per thread is the 16-bit path");
  const uint32_t lb = xcd_block(blockIdx.x, gridDim.x);
  const uint32_t bxi = lb % bpr, rowid = lb / bpr;
  const int y = (int)(rowid % (uint32_t)k.ny), z = (int)(rowid / (uint32_t)k.ny);
  const uint32_t tpr = (uint32_t)k.nx / 2;                      // words per row (nx even)
  const uint32_t t = bxi * blockDim.x + threadIdx.x;
  if (t >= tpr) return;
  const uint32_t tm = t == 0 ? tpr - 1 : t - 1, tp = t + 1 == tpr ? 0 : t + 1;
  Upstream u;
  upstream((int)(2 * t), y, z, k, u);
  const PairWords p = pair_words(t, tm, tp);
  uint32_t w[27];
  gather_pair<ST>(pull_groups(src, u), p, w);
  uint32_t o[27];
  collide_pair<ST, CORR, RAW, HI>(w, force, ((int64_t)z * k.ny + y) * k.nx, 2 * t, k, o);
  store_pair_own<ST>(own_groups(dst, u), store_offset(p.xw[1]), o);
}

// Full corrections (CORR 3) with two nodes per thread: the pair gather and word
// stores of k_step_pair, the density gradient of both nodes from the block's
// column sums (density_gradient_pair_block), and, if drho_out is not NULL, both
// nodes' density deviations.  Same values as k_step<ST, 3, 0> bit for bit.
template <int ST, bool RAW>
__global__ __launch_bounds__(256) void k_step_full_pair(const typename Store<ST>::T* __restrict__ src,
                                                        typename Store<ST>::T* __restrict__ dst,
                                                        const float* __restrict__ force,
                                                        const float* __restrict__ grad_src,
                                                        float* __restrict__ drho_out, Consts k, uint32_t bpr) {
  static_assert(ST != 0, "two nodes per thread is the 16-bit path");
  const uint32_t lb = xcd_block(blockIdx.x, gridDim.x);
  const uint32_t bxi = lb % bpr, rowid = lb / bpr;
  int y, z;
  tiled_row(rowid, (uint32_t)k.ytile, k, y, z);
  const uint32_t tpr = (uint32_t)k.nx / 2;
  const uint32_t t = bxi * blockDim.x + threadIdx.x;
  __shared__ float lds[3][258];
  float g[2][3];
  density_gradient_pair_block(grad_src, (int)(2 * t), y, z, t < tpr, k, lds, g);
  if (t >= tpr) return;
  const uint32_t tm = t == 0 ? tpr - 1 : t - 1, tp = t + 1 == tpr ? 0 : t + 1;
  Upstream u;
  upstream((int)(2 * t), y, z, k, u);
  const PairWords p = pair_words(t, tm, tp);
  uint32_t w[27];
  gather_pair<ST>(pull_groups(src, u), p, w);
  const int64_t nrow = ((int64_t)z * k.ny + y) * k.nx;
  PairWord<ST> pw[27];
#pragma unroll
  for (int h = 0; h < 2; ++h) {
    float df[27];
#pragma unroll
    for (int a = 0; a < 27; ++a) df[a] = decode_scale<ST>(word_half<ST>(w[a], h), wclass(a), k);
    float fx, fy, fz;
    node_force(force, nrow, 2 * t + h, k, fx, fy, fz);
    float out[27];
    collide_fenced<3, RAW, false, false>(df, fx, fy, fz, k, out, g[h][0], g[h][1], g[h][2]);
    if (drho_out != nullptr) st_off(drho_out + nrow, 2 * t + h, low_moments(df).m000);
    if constexpr (ST == 3) {
      const uint32_t r16 = sr_bits((uint32_t)nrow + 2 * t + h, k.seq_hash);
#pragma unroll
      for (int a = 0; a < 27; ++a) pw[a].put(h, out[a], r16);
    } else {
#pragma unroll
      for (int a = 0; a < 27; ++a) pw[a].put(h, encode_scale<ST>(out[a], wclass(a), k));
    }
  }
  uint32_t o[27];
#pragma unroll
  for (int a = 0; a < 27; ++a) o[a] = pw[a].bits();
  store_pair_own<ST>(own_groups(dst, u), store_offset(p.xw[1]), o);
}

// ------------------------------------------------------------------ step, AA layout
// One buffer updated in place.  Even steps (ODD = false): node x reads its own
// slots (a, x), collides and writes f~_a to (opp(a), x).  Odd steps: f_a(x) is
// read from (opp(a), x - ebar_a), or from (a, x) when x - ebar_a lies beyond a
// wall, and f~_a is written to (a, x + ebar_a), or to (opp(a), x) when
// x + ebar_a lies beyond a wall.  Within a step every slot is read and written
// by one node only, so the update needs no second buffer.  After an even
// number of steps slot (a, x) holds f_a(x) again.  Without walls through row
// addresses (any state size); with walls through 32-bit offsets from the start
// of the state (below 4 GiB).
// Chunk group bases of an AA step: the node's own row (even steps) or the
// rows of aa_odd_groups (odd steps); unused with walls.
template <bool ODD, typename T>
__device__ __forceinline__ GroupBases<T> aa_groups(T* state, const Upstream& u) {
  if constexpr (ODD) return aa_odd_groups(state, u);
  else return own_groups(state, u);
}

template <int ST, bool ODD, bool WALLS, int I = 0>
__device__ __forceinline__ void gather_aa(const typename Store<ST>::T* __restrict__ src,
                                          const GroupBases<typename Store<ST>::T>& b, const Upstream& u,
                                          const WallFlags& w, const Consts& k, float (&df)[27]) {
  constexpr int A = issue_dir(I);
  constexpr int opp = opposite_of(A);
  // even steps read the node's own slots (no line shared between waves): all non-temporal;
  // odd steps as the two-buffer gather
  constexpr bool NT = !ODD || kEx[A] == 0 || LBM_GATHER_NT == 1;
  typename Store<ST>::T v;
  if constexpr (!ODD) {
    v = ld_pop<NT>(chunk_ptr<A>(b), u.xo[1]);
  } else if constexpr (WALLS) {
    v = ld_pop<NT>(src, pulls_through_wall<A>(w) ? own_slot32<A>(u) : upstream_slot32<A, opp>(u));
  } else {
    v = ld_pop<NT>(b.g[group_of(A)] + (1 - kEx[A]) * kB, u.xo[kEx[A] + 1]);
  }
  const float f = Store<ST>::load_val(v);
  df[A] = decode_scale<ST>(f, wclass(A), k);
  if constexpr (I + 1 < 27) gather_aa<ST, ODD, WALLS, I + 1>(src, b, u, w, k, df);
}

template <int ST, bool ODD, bool WALLS, int I = 0>
__device__ __forceinline__ void store_aa(typename Store<ST>::T* __restrict__ dst,
                                         const GroupBases<typename Store<ST>::T>& b, const Upstream& u,
                                         const WallFlags& w, const Consts& k, const float (&out)[27],
                                         uint32_t r16) {
  constexpr int A = issue_dir(I);
  constexpr int opp = opposite_of(A);
  const typename Store<ST>::T v = pack_rounded<ST>(encode_scale<ST>(out[A], wclass(A), k), r16);
  if constexpr (!ODD) {
    st_off_nt(chunk_ptr<opp>(b), u.xo[1], v);
  } else if constexpr (WALLS) {
    // x + ebar_A lies beyond a wall exactly when opp(A) pulls through one
    const uint32_t idx = pulls_through_wall<opp>(w) ? own_slot32<opp>(u) : upstream_slot32<opp, A>(u);
    if constexpr (kEx[A] == 0) st_off_nt(dst, idx, v);
    else st_off(dst, idx, v);
  } else {
    // shifted by one node along x for 18 directions: plain stores, partial lines merge in L2;
    // the 9 with ebar_x = 0 write whole lines: non-temporal stores
    global_t<typename Store<ST>::T>* p = b.g[8 - group_of(A)] + (kEx[A] + 1) * kB;
    if constexpr (kEx[A] == 0) st_off_nt(p, u.xo[1], v);
    else st_off(p, u.xo[1 - kEx[A]], v);
  }
  if constexpr (I + 1 < 27) store_aa<ST, ODD, WALLS, I + 1>(dst, b, u, w, k, out, r16);
}

template <int ST, int CORR, bool ODD, bool WALLS, bool RAW, bool HI>
__global__ __launch_bounds__(256, step_waves(ST, CORR)) void k_step_aa(typename Store<ST>::T* __restrict__ state,
                                                                       const float* __restrict__ force, Consts k,
                                                                       uint32_t bpr) {
  const uint32_t lb = xcd_block(blockIdx.x, gridDim.x);
  const uint32_t bxi = lb % bpr, rowid = lb / bpr;
  const int y = (int)(rowid % (uint32_t)k.ny), z = (int)(rowid / (uint32_t)k.ny);
  const int x = (int)(bxi * blockDim.x + threadIdx.x);
  if (x >= k.nx) return;
  Upstream u;
  upstream(x, y, z, k, u);
  WallFlags w{};
  if constexpr (WALLS) w = wall_flags(x, y, z, k);
  // group bases: every even step (own slots) and the odd steps without walls
  // (the odd steps with walls address through 32-bit offsets from the state)
  const GroupBases<typename Store<ST>::T> b = aa_groups<ODD>(state, u);
  float df[27];
  gather_aa<ST, ODD, WALLS>(state, b, u, w, k, df);
  float fx, fy, fz;
  node_force(force, ((int64_t)z * k.ny + y) * k.nx, (uint32_t)x, k, fx, fy, fz);
  float out[27];
  collide_fenced<CORR, RAW, HI, ST == 0 || HI>(df, fx, fy, fz, k, out);
  if constexpr (ST == 0) conserve(df, fx, fy, fz, k, out);
  if constexpr (WALLS) {
    if (k.moving) moving_wall_terms(x, y, z, k.rho0 + low_moments(df).m000, k, out);
  }
  const uint32_t node = ((uint32_t)z * (uint32_t)k.ny + (uint32_t)y) * (uint32_t)k.nx + (uint32_t)x;
  store_aa<ST, ODD, WALLS>(state, b, store_upstream(u), w, k, out, node_sr_bits<ST>(node, k));
}

// 16-bit AA step with two x-adjacent nodes per thread (periodic grids, even nx;
// the pairing of k_step_pair).  Even steps read and write whole words of the
// node pair's own slots.  Odd steps gather like k_step_pair from the opposite
// directions' chunks; their x-shifted outputs land in words that two threads
// share, so those go out as 2-byte stores.
template <int ST, bool ODD, int I = 0>
__device__ __forceinline__ void gather_aa_pair(const GroupBases<typename Store<ST>::T>& b, const PairWords& p,
                                               uint32_t (&w)[27]) {
  constexpr int A = issue_dir(I);
  if constexpr (!ODD) w[A] = ld_off_nt(words(chunk_ptr<A>(b)), p.xw[1]);
  else w[A] = pair_gather_word<A>(b.g[group_of(A)] + (1 - kEx[A]) * kB, p);
  if constexpr (I + 1 < 27) gather_aa_pair<ST, ODD, I + 1>(b, p, w);
}

// WS (odd steps, every wave within one row: nx a multiple of 128): the x-shifted
// outputs as whole 32-bit words assembled across lanes instead of 2-byte stores.
template <int ST, bool ODD, bool WS, int I = 0>
__device__ __forceinline__ void store_aa_pair(const GroupBases<typename Store<ST>::T>& b, const PairWords& p,
                                              const uint32_t (&o)[27]) {
  constexpr int A = issue_dir(I);
  constexpr int ex = kEx[A];
  if constexpr (!ODD) {
    st_off_nt(words(chunk_ptr<opposite_of(A)>(b)), p.xw[1], o[A]);
  } else {
    // f~_A of nodes 2t, 2t + 1 goes to (A, x + ebar_A): row y + ey, z + ez
    global_t<typename Store<ST>::T>* row = b.g[8 - group_of(A)] + (ex + 1) * kB;
    if constexpr (ex == 0) {
      st_off_nt(words(row), p.xw[1], o[A]);
    } else {
      global_t<unsigned short>* base = reinterpret_cast<global_t<unsigned short>*>(row);
      const uint32_t lo = o[A] & 0xffffu, hi = o[A] >> 16;
      if constexpr (WS) {
        // Whole words: the half that completes this lane's word comes from the
        // neighbouring lane (a wavefront shift); the two halves without a partner in
        // the wave (lane 0's and lane 63's) are 2-byte stores of one instruction.
        const uint32_t lane = threadIdx.x & 63u;
        if constexpr (ex > 0) {  // word t = (node 2t: hi of lane - 1, node 2t + 1: lo of this lane)
          const uint32_t prev = (uint32_t)__builtin_amdgcn_mov_dpp((int)hi, 0x138, 0xf, 0xf, false);
          if (lane != 0) st_off(words(row), p.xw[1], prev | (lo << 16));
          if (lane == 0 || lane == 63)
            st_off<unsigned short>(base, lane == 0 ? 2 * p.xw[1] + 1 : 2 * p.xw[0],
                                   (unsigned short)(lane == 0 ? lo : hi));
        } else {                 // word t = (node 2t: hi of this lane, node 2t + 1: lo of lane + 1)
          const uint32_t next = (uint32_t)__builtin_amdgcn_mov_dpp((int)lo, 0x130, 0xf, 0xf, false);
          if (lane != 63) st_off(words(row), p.xw[1], hi | (next << 16));
          if (lane == 0 || lane == 63)
            st_off<unsigned short>(base, lane == 63 ? 2 * p.xw[1] : 2 * p.xw[2] + 1,
                                   (unsigned short)(lane == 63 ? hi : lo));
        }
      } else if constexpr (ex > 0) {                              // nodes 2t + 1, 2t + 2
        st_off<unsigned short>(base, 2 * p.xw[1] + 1, (unsigned short)lo);
        st_off<unsigned short>(base, 2 * p.xw[0], (unsigned short)hi);
      } else {                                                   // nodes 2t - 1, 2t
        st_off<unsigned short>(base, 2 * p.xw[2] + 1, (unsigned short)lo);
        st_off<unsigned short>(base, 2 * p.xw[1], (unsigned short)hi);
      }
    }
  }
  if constexpr (I + 1 < 27) store_aa_pair<ST, ODD, WS, I + 1>(b, p, o);
}

template <int ST, int CORR, bool ODD, bool RAW, bool HI, bool WS>
__global__ __launch_bounds__(256) void k_step_aa_pair(typename Store<ST>::T* __restrict__ state,
                                                      const float* __restrict__ force, Consts k, uint32_t bpr) {
  static_assert(ST != 0, "two nodes per thread is the 16-bit path");
  const uint32_t lb = xcd_block(blockIdx.x, gridDim.x);
  const uint32_t bxi = lb % bpr, rowid = lb / bpr;
  const int y = (int)(rowid % (uint32_t)k.ny), z = (int)(rowid / (uint32_t)k.ny);
  const uint32_t tpr = (uint32_t)k.nx / 2;
  const uint32_t t = bxi * blockDim.x + threadIdx.x;
  if (t >= tpr) return;
  const uint32_t tm = t == 0 ? tpr - 1 : t - 1, tp = t + 1 == tpr ? 0 : t + 1;
  Upstream u;
  upstream((int)(2 * t), y, z, k, u);
  const PairWords p = pair_words(t, tm, tp);
  const GroupBases<typename Store<ST>::T> b = aa_groups<ODD>(state, u);
  uint32_t w[27];
  gather_aa_pair<ST, ODD>(b, p, w);
  uint32_t o[27];
  collide_pair<ST, CORR, RAW, HI>(w, force, ((int64_t)z * k.ny + y) * k.nx, 2 * t, k, o);
  PairWords ps;
#pragma unroll
  for (int i = 0; i < 3; ++i) ps.xw[i] = store_offset(p.xw[i]);
  store_aa_pair<ST, ODD, WS>(b, ps, o);
}

// Density deviation of every node of a state: the same gather and the same
// FP32 sum as the step, so the value is bit-identical to the step's.
template <int ST, int WALLS>
__global__ __launch_bounds__(256) void k_density(const typename Store<ST>::T* __restrict__ src,
                                                 float* __restrict__ drho, Consts k, uint32_t bpr) {
  const uint32_t lb = xcd_block(blockIdx.x, gridDim.x);
  const uint32_t bxi = lb % bpr, rowid = lb / bpr;
  const int y = (int)(rowid % (uint32_t)k.ny), z = (int)(rowid / (uint32_t)k.ny);
  const int x = (int)(bxi * blockDim.x + threadIdx.x);
  if (x >= k.nx) return;
  Upstream u;
  upstream(x, y, z, k, u);
  float df[27];
  gather_node<ST, WALLS>(src, u, x, y, z, k, df);
  st_off(drho + ((int64_t)z * k.ny + y) * k.nx, (uint32_t)x, low_moments(df).m000);
}

// ------------------------------------------------------------------ streaming only
// The step's gather and store with the collision left out: f_a(x, t+1) =
// f_a(x - ebar_a, t), or f_abar(x, t) across a stationary wall.  It moves the
// step's bytes in the step's access pattern (same kernel shape, block size and
// occupancy cap), so its rate is the ceiling of that pattern.  16-bit values
// pass through unchanged (decode and encode scale by a power of two).
template <int ST, int WALLS>
__global__ __launch_bounds__(256) void k_stream(const typename Store<ST>::T* __restrict__ src,
                                                typename Store<ST>::T* __restrict__ dst, Consts k, uint32_t bpr) {
  const uint32_t lb = xcd_block(blockIdx.x, gridDim.x);
  const uint32_t bxi = lb % bpr, rowid = lb / bpr;
  const int y = (int)(rowid % (uint32_t)k.ny), z = (int)(rowid / (uint32_t)k.ny);
  const int x = (int)(bxi * blockDim.x + threadIdx.x);
  if (x >= k.nx) return;
  Upstream u;
  upstream(x, y, z, k, u);
  float df[27];
  gather_node<ST, WALLS>(src, u, x, y, z, k, df);
  const uint32_t node = ((uint32_t)z * (uint32_t)k.ny + (uint32_t)y) * (uint32_t)k.nx + (uint32_t)x;
  store_own<ST>(own_groups(dst, u), store_offset(u.xo[1]), df, k, node_sr_bits<ST>(node, k));
}

// Streaming only in the pair step's shape (16-bit periodic storage, even nx, two
// nodes per thread): the pair gather and word stores without the collisions.
template <int ST>
__global__ __launch_bounds__(256) void k_stream_pair(const typename Store<ST>::T* __restrict__ src,
                                                     typename Store<ST>::T* __restrict__ dst, Consts k, uint32_t bpr) {
  static_assert(ST != 0, "two nodes per thread is the 16-bit path");
  const uint32_t lb = xcd_block(blockIdx.x, gridDim.x);
  const uint32_t bxi = lb % bpr, rowid = lb / bpr;
  const int y = (int)(rowid % (uint32_t)k.ny), z = (int)(rowid / (uint32_t)k.ny);
  const uint32_t tpr = (uint32_t)k.nx / 2;
  const uint32_t t = bxi * blockDim.x + threadIdx.x;
  if (t >= tpr) return;
  const uint32_t tm = t == 0 ? tpr - 1 : t - 1, tp = t + 1 == tpr ? 0 : t + 1;
  Upstream u;
  upstream((int)(2 * t), y, z, k, u);
  const PairWords p = pair_words(t, tm, tp);
  uint32_t w[27];
  gather_pair<ST>(pull_groups(src, u), p, w);
  store_pair_own<ST>(own_groups(dst, u), store_offset(p.xw[1]), w);
}

// ------------------------------------------------------------------ launchers
// Gather path: 0 periodic (row addresses, any size); 1 walls, 32-bit offsets
// across the whole state (below 4 GiB); 2 general, 64-bit slots (walls above
// 4 GiB).  lbm_create's LBM_GATHER_KIND override selects a more general path
// where it is valid (tests run the 64-bit path on small grids that way).
static inline int gather_kind(const lbm_handle& h) {
  const bool walls = h.k.bb_x || h.k.bb_y || h.k.bb_z;
  const bool fits32 = 27ull * (uint64_t)h.stride * h.elem < (1ull << 32);
  int kind = !walls ? 0 : (fits32 ? 1 : 2);
  if (h.force_kind > kind && (h.force_kind == 2 || fits32)) kind = h.force_kind;
  return kind;
}

template <int ST, bool HI>
static hipError_t launch_step_t(const lbm_handle& h, const void* src, void* dst, const float* force,
                                const float* grad_src, float* drho_out, hipStream_t st) {
  using T = typename Store<ST>::T;
  const int block = h.p.corr == LBM_CORR_FULL ? h.block : h.block_step;
  const uint32_t bpr = (uint32_t)((h.p.nx + block - 1) / block);
  const int64_t nb = (int64_t)bpr * h.p.ny * h.p.nz;
  if (nb > 0x7fffffffLL) return hipErrorInvalidConfiguration;
  const T* s = (const T*)src;
  T* d = (T*)dst;
  const int kind = gather_kind(h);
  // two nodes per thread: the unit higher-order rate only (with a general rate the
  // two collisions of a thread share rate-dependent terms, which the compiler then
  // fuses differently from the one-node kernel, so the results would differ in
  // the last bit)
  if constexpr (ST != 0 && !HI) {
    if (kind == 0 && h.pairs && h.p.corr == LBM_CORR_FULL && h.p.nx % 2 == 0) {
      constexpr int pblock = 128;                               // lds of 2 * 128 + 2 columns
      const uint32_t pbpr = (uint32_t)((h.p.nx / 2 + pblock - 1) / pblock);
      const int64_t pnb = (int64_t)pbpr * h.p.ny * h.p.nz;
      if (pnb > 0x7fffffffLL) return hipErrorInvalidConfiguration;
      if (h.p.moments == LBM_RAW)
        hipLaunchKernelGGL((k_step_full_pair<ST, true>), dim3((unsigned)pnb), dim3(pblock), 0, st, s, d, force,
                           grad_src, drho_out, h.k, pbpr);
      else
        hipLaunchKernelGGL((k_step_full_pair<ST, false>), dim3((unsigned)pnb), dim3(pblock), 0, st, s, d, force,
                           grad_src, drho_out, h.k, pbpr);
      return hipGetLastError();
    }
    if (kind == 0 && h.pairs && h.p.corr != LBM_CORR_FULL && h.p.nx % 2 == 0) {
      constexpr int pblock = 128;                               // measured best of 64 / 128 / 256
      const uint32_t pbpr = (uint32_t)((h.p.nx / 2 + pblock - 1) / pblock);
      const int64_t pnb = (int64_t)pbpr * h.p.ny * h.p.nz;
      if (pnb > 0x7fffffffLL) return hipErrorInvalidConfiguration;
      const dim3 pgrid((unsigned)pnb), pblk(pblock);
#define CLBM_PAIR(C, R) \
  hipLaunchKernelGGL((k_step_pair<ST, C, R, HI>), pgrid, pblk, (unsigned)h.pair_lds, st, s, d, force, h.k, pbpr)
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
  hipLaunchKernelGGL((k_step<ST, C, W, R, HI>), grid, blk, lds, st, s, d, force, grad_src, drho_out, h.k, bpr)
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
  const T* s = (const T*)src;
  const dim3 grid((unsigned)nb), blk(block);
  switch (h.k.aa ? 2 : gather_kind(h)) {  // the AA layout keeps natural order: general slot rule
    case 0: hipLaunchKernelGGL((k_density<ST, 0>), grid, blk, 0, st, s, drho, h.k, bpr); break;
    case 1: hipLaunchKernelGGL((k_density<ST, 1>), grid, blk, 0, st, s, drho, h.k, bpr); break;
    default: hipLaunchKernelGGL((k_density<ST, 2>), grid, blk, 0, st, s, drho, h.k, bpr); break;
  }
  return hipGetLastError();
}

template <int ST>
static hipError_t launch_stream_t(const lbm_handle& h, const void* src, void* dst, hipStream_t st) {
  using T = typename Store<ST>::T;
  const int block = h.block_step;
  const uint32_t bpr = (uint32_t)((h.p.nx + block - 1) / block);
  const int64_t nb = (int64_t)bpr * h.p.ny * h.p.nz;
  if (nb > 0x7fffffffLL) return hipErrorInvalidConfiguration;
  const T* s = (const T*)src;
  T* d = (T*)dst;
  if constexpr (ST != 0) {  // the launch shape of the pair step
    if (gather_kind(h) == 0 && h.pairs && h.p.nx % 2 == 0) {
      constexpr int pblock = 128;
      const uint32_t pbpr = (uint32_t)((h.p.nx / 2 + pblock - 1) / pblock);
      const int64_t pnb = (int64_t)pbpr * h.p.ny * h.p.nz;
      if (pnb > 0x7fffffffLL) return hipErrorInvalidConfiguration;
      hipLaunchKernelGGL((k_stream_pair<ST>), dim3((unsigned)pnb), dim3(pblock), (unsigned)h.pair_lds, st, s, d,
                         h.k, pbpr);
      return hipGetLastError();
    }
  }
  const dim3 grid((unsigned)nb), blk(block);
  const unsigned lds = (unsigned)h.step_lds;
  switch (gather_kind(h)) {
    case 0: hipLaunchKernelGGL((k_stream<ST, 0>), grid, blk, lds, st, s, d, h.k, bpr); break;
    case 1: hipLaunchKernelGGL((k_stream<ST, 1>), grid, blk, lds, st, s, d, h.k, bpr); break;
    default: hipLaunchKernelGGL((k_stream<ST, 2>), grid, blk, lds, st, s, d, h.k, bpr); break;
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
  T* s = (T*)state;
  const bool walls = h.k.bb_x || h.k.bb_y || h.k.bb_z;
  if constexpr (ST != 0 && !HI) {  // as in the two-buffer step
    if (!walls && h.pairs && h.p.nx % 2 == 0) {
      constexpr int pblock = 128;
      const uint32_t pbpr = (uint32_t)((h.p.nx / 2 + pblock - 1) / pblock);
      const int64_t pnb = (int64_t)pbpr * h.p.ny * h.p.nz;
      if (pnb > 0x7fffffffLL) return hipErrorInvalidConfiguration;
      const dim3 pgrid((unsigned)pnb), pblk(pblock);
      // whole-word stores of the odd step need every wave inside one row (lane 0 starts a
      // 64-pair segment): nx a multiple of 128
      const bool ws = h.p.nx % 128 == 0;
#define CLBM_AAP(C, O, R)                                                                                     \
  if (O && ws)                                                                                                \
    hipLaunchKernelGGL((k_step_aa_pair<ST, C, true, R, HI, true>), pgrid, pblk, (unsigned)h.pair_lds, st, s,   \
                       force, h.k, pbpr);                                                                     \
  else                                                                                                        \
    hipLaunchKernelGGL((k_step_aa_pair<ST, C, O, R, HI, false>), pgrid, pblk, (unsigned)h.pair_lds, st, s,     \
                       force, h.k, pbpr)
#define CLBM_AAP_R(C, O) if (h.p.moments == LBM_RAW) { CLBM_AAP(C, O, true); } else { CLBM_AAP(C, O, false); }
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
  hipLaunchKernelGGL((k_step_aa<ST, C, O, W, R, HI>), grid, blk, (unsigned)h.step_lds, st, s, force, h.k, bpr)
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

template <int ST>
hipError_t StepKernels<ST>::stream(const lbm_handle& h, const void* src, void* dst, hipStream_t st) {
  return launch_stream_t<ST>(h, src, dst, st);
}

}  // namespace clbm
