// Device-side building blocks of the cuboid D3Q27 central-moment step (gfx950).
//
// Layout: a state is blocked.  Each x-row of the grid is padded to a multiple
// of kB nodes and cut into blocks of kB consecutive nodes; a block stores the
// 27 directions (eq. 1a-c) of its nodes as 27 chunks of kB elements.  An
// element is a population slot holding the deviation (f - w_alpha rho0)
// scaled by sigma_alpha (1 for FP32 storage).  Pull scheme: the step at node x
// gathers f_alpha(x) from slot (alpha, x - ebar_alpha), or from
// (opposite(alpha), x) when x - ebar_alpha lies beyond a bounce-back wall
// (Sec. 4, stationary wall), and writes its post-collision populations to the
// slots (alpha, x) of the other buffer.
#pragma once

#include <hip/hip_runtime.h>
#include <hip/hip_fp16.h>
#include <hip/hip_bf16.h>
#include <stdint.h>

#include <type_traits>

namespace clbm {

// eq. 1a-c: integer velocity components; e = (ebar_x, r ebar_y, s ebar_z).
constexpr int kEx[27] = {0, 1, -1, 0, 0, 0, 0, 1, -1, 1, -1, 1, -1, 1, -1, 0, 0, 0, 0, 1, -1, 1, -1, 1, -1, 1, -1};
constexpr int kEy[27] = {0, 0, 0, 1, -1, 0, 0, 1, 1, -1, -1, 0, 0, 0, 0, 1, -1, 1, -1, 1, 1, -1, -1, 1, 1, -1, -1};
constexpr int kEz[27] = {0, 0, 0, 0, 0, 1, -1, 0, 0, 0, 0, 1, 1, -1, -1, 1, 1, -1, -1, 1, 1, 1, 1, -1, -1, -1, -1};

constexpr int opposite_of(int a) {
  for (int b = 0; b < 27; ++b)
    if (kEx[b] == -kEx[a] && kEy[b] == -kEy[a] && kEz[b] == -kEz[a]) return b;
  return -1;
}

// Weight class of a direction: which of its components are non-zero.  The
// weights of eq. 9-10 are products of per-axis factors that depend only on
// |ebar_d|, so the eight classes carry every distinct weight (and storage scale).
constexpr int wclass(int a) { return (kEx[a] != 0) + 2 * (kEy[a] != 0) + 4 * (kEz[a] != 0); }

// Direction with components (i-1, j-1, k-1), i, j, k in {0, 1, 2}.
constexpr int dir_of(int i, int j, int k) {
  for (int a = 0; a < 27; ++a)
    if (kEx[a] == i - 1 && kEy[a] == j - 1 && kEz[a] == k - 1) return a;
  return -1;
}

// Per-launch constants, passed by value as a kernel argument.
struct Consts {
  int nx, ny, nz;
  int bb_x, bb_y, bb_z;    // 1 = halfway bounce-back walls on that axis
  int moving;              // bit f set = face f moves (momentum-augmented bounce-back)
  int ytile;               // rows per y-tile of the full-correction step's row order (divides ny)
  int aa;                  // 1 = AA layout: between calls slot (a, x) holds f_a(x) (natural order)
  float wall_u[6][3];      // face velocities, faces x-, x+, y-, y+, z-, z+
  int64_t row_slots;       // elements of one grid row of a state (27 kB ceil(nx / kB))
  int64_t n;               // nodes
  float rho0, cs2, r, s;
  float omega_nu, omega_xi;
  float fx, fy, fz;        // uniform force
  float c2[3];             // squared particle speeds 1, r^2, s^2
  float ic[3], ic2[3];     // 1/c, 1/c^2 per axis
  float w0c[3], w0s[3];    // rest weights per axis: centre 1 - cs2/c^2, side cs2/(2 c^2)
  float sigma[8];          // storage scale per weight class (wclass)
  float inv_sigma[8];
  float omega_hi;          // rate of the moments of order >= 3
  int hi;                  // 1 = omega_hi != 1 (kernels with the general higher-order rate)
  uint32_t seq_hash;       // per-step key of the stochastic rounding (BF16-SR storage)
};

// FP64 copies for the one-time conversions (init, import, export).
struct ConstsD {
  double rho0, cs2;
  double ic[3], ic2[3];
  double w0c[3], w0s[3];
  double w[27];            // w_alpha = product of the per-axis rest weights
};

// ----------------------------------------------------------------- storage
template <int ST> struct Store;

template <> struct Store<0> {
  using T = float;
  static __device__ __forceinline__ float load(const T* p) { return *p; }
  static __device__ __forceinline__ float load_val(T v) { return v; }
  static __device__ __forceinline__ T pack(float v) { return v; }
};

// 16-bit formats also convert from the raw 16 bits (the pair steps keep two
// nodes' values in one 32-bit word), with the same conversion.
template <> struct Store<1> {
  using T = __half;
  static __device__ __forceinline__ float load(const T* p) { return __half2float(*p); }
  static __device__ __forceinline__ float load_val(T v) { return __half2float(v); }
  static __device__ __forceinline__ T pack(float v) { return __float2half_rn(v); }
  static __device__ __forceinline__ float from_bits(uint32_t b) {
    return __half2float(__builtin_bit_cast(__half, (unsigned short)b));
  }
};

template <> struct Store<2> {
  using T = __hip_bfloat16;
  static __device__ __forceinline__ float load(const T* p) { return __bfloat162float(*p); }
  static __device__ __forceinline__ float load_val(T v) { return __bfloat162float(v); }
  static __device__ __forceinline__ T pack(float v) { return __float2bfloat16(v); }
  static __device__ __forceinline__ float from_bits(uint32_t b) {
    return __bfloat162float(__builtin_bit_cast(__hip_bfloat16, (unsigned short)b));
  }
};

// BF16 with stochastic rounding (LBM_BF16_SR): the BF16 format, read like
// Store<2>; the step's stores round up with probability equal to the discarded
// fraction (bf16_sr_bits), so the rounding is unbiased even where a slowly
// changing flow would round every step the same way.  One-time conversions
// (init, import) round to nearest like Store<2>.
template <> struct Store<3> : Store<2> {};

template <int ST>
constexpr bool kBf16 = ST == 2 || ST == 3;

// Only FP16 storage scales the deviations (sigma_a, a power of two near 1/w_a,
// keeps them in its normal range).  FP32 and BF16 have the FP32 exponent range,
// so they store the deviations unscaled (sigma = 1, a power of two changes no
// rounding) and their kernels skip the scaling.
template <int ST>
constexpr bool kScaled = ST == 1;

template <int ST>
__device__ __forceinline__ float decode_scale(float v, int cls, const Consts& k) {
  if constexpr (kScaled<ST>) return v * k.inv_sigma[cls];
  else return v;
}

template <int ST>
__device__ __forceinline__ float encode_scale(float v, int cls, const Consts& k) {
  if constexpr (kScaled<ST>) return v * k.sigma[cls];
  else return v;
}

// The two halves of a 32-bit word of two 16-bit values (first node in the low
// half) as floats; BF16 is the upper half of an FP32 pattern, so its decode is
// a shift or a mask.
template <int ST>
__device__ __forceinline__ float word_half(uint32_t w, int h) {
  if constexpr (kBf16<ST>) return __builtin_bit_cast(float, h ? (w & 0xffff0000u) : (w << 16));
  else return Store<ST>::from_bits(h ? w >> 16 : w & 0xffffu);
}

// 16 random bits per node and step for the stochastic rounding: a published
// integer hash (Wellons' "lowbias32" finalizer) of the node index mixed with the
// per-step key k.seq_hash.  Counter-based, so a step recomputed from the same
// state with the same step counter rounds identically.
__device__ __forceinline__ uint32_t sr_bits(uint32_t node, uint32_t seq_hash) {
  uint32_t v = node ^ seq_hash;
  v ^= v >> 16;
  v *= 0x7feb352du;
  v ^= v >> 15;
  v *= 0x846ca68bu;
  v ^= v >> 16;
  return v & 0xffffu;
}

// FP32 pattern whose upper 16 bits are x rounded stochastically to BF16: the
// lower 16 bits f are added to r = f ^ r16, which is uniform on [0, 2^16) when
// r16 is, so the carry into the upper half happens with probability f / 2^16
// (sign-magnitude: the magnitude rounds up or down, the sign is kept).
__device__ __forceinline__ uint32_t bf16_sr_bits(float x, uint32_t r16) {
  const uint32_t b = __builtin_bit_cast(uint32_t, x);
  return b + ((b & 0xffffu) ^ r16);
}

template <int ST>
__device__ __forceinline__ typename Store<ST>::T pack_rounded(float v, uint32_t r16) {
  if constexpr (ST == 3) return __builtin_bit_cast(typename Store<ST>::T, (unsigned short)(bf16_sr_bits(v, r16) >> 16));
  else return Store<ST>::pack(v);
}

// One direction's values of two x-adjacent nodes in the 32-bit word the pair
// steps store (first node in the low half), filled one node at a time with the
// same rounding as Store<ST>::pack.  FP16 converts each value as it comes (the
// high half is written in place); BF16 keeps the first value and converts both
// with one two-value instruction.
template <int ST> struct PairWord;

template <> struct PairWord<1> {
  typedef _Float16 h2 __attribute__((ext_vector_type(2)));
  h2 v;
  __device__ __forceinline__ void put(int h, float x) {
    if (h) v.y = (_Float16)x;
    else v.x = (_Float16)x;
  }
  __device__ __forceinline__ uint32_t bits() const { return __builtin_bit_cast(uint32_t, v); }
};

template <> struct PairWord<3> {
  uint32_t first, word;
  __device__ __forceinline__ void put(int h, float x, uint32_t r16) {
    const uint32_t b = bf16_sr_bits(x, r16);
    if (h) word = (b & 0xffff0000u) | (first >> 16);
    else first = b;
  }
  __device__ __forceinline__ uint32_t bits() const { return word; }
};

template <> struct PairWord<2> {
  typedef float f2 __attribute__((ext_vector_type(2)));
  typedef __bf16 b2 __attribute__((ext_vector_type(2)));
  float first;
  uint32_t word;
  __device__ __forceinline__ void put(int h, float x) {
    if (h) word = __builtin_bit_cast(uint32_t, __builtin_convertvector((f2){first, x}, b2));
    else first = x;
  }
  __device__ __forceinline__ uint32_t bits() const { return word; }
};

// ----------------------------------------------------------------- state layout
// Nodes per block.  A wave of 64 lanes reads one direction of 64 (one node per
// lane) or 128 (two per lane) consecutive nodes as whole lines of one chunk,
// and a node's 27 slots lie in one block instead of 27 separate arrays; at
// 512x512x256 the pull pattern moved 6.07 TB/s this way against 5.54 with
// one array per direction.
constexpr int kB = 128;

// Chunk of direction a within a block: grouped by upstream row, the three
// directions with the same (ebar_y, ebar_z) side by side in the order
// ebar_x = -1, 0, +1, so a node's pulls from one row are adjacent in memory.
// The opposite direction's chunk is 26 - chunk_of(a).
// Group of upstream row (ebar_y, ebar_z), y-major (a z-major order of the nine
// groups measured the same at 512x512x256, FP32 and FP16).
constexpr int group_index(int ey, int ez) { return 3 * (ey + 1) + (ez + 1); }
constexpr int group_ey(int g) { return g / 3 - 1; }
constexpr int group_ez(int g) { return g % 3 - 1; }
constexpr int chunk_of(int a) { return 3 * group_index(kEy[a], kEz[a]) + (kEx[a] + 1); }

// Order in which the gathers and stores issue the 27 directions: direction
// order (memory order, chunk by chunk, measured the same on the FP32 and FP16
// steps at 512x512x256).
constexpr int issue_dir(int i) { return i; }

// Element offset of node x within its row: (x / kB) 27 kB + x % kB.
__device__ __forceinline__ uint32_t xoff(uint32_t x) { return (x / kB) * (27u * kB) + x % kB; }

// First element of grid row (y, z).
__device__ __forceinline__ int64_t row_start(int y, int z, const Consts& k) {
  return ((int64_t)z * k.ny + y) * k.row_slots;
}

// Element of slot (a, x, y, z).
template <int A>
__device__ __forceinline__ int64_t slot_of(int x, int y, int z, const Consts& k) {
  return row_start(y, z, k) + (int64_t)(chunk_of(A) * kB) + (int64_t)xoff((uint32_t)x);
}

struct NodeCoord {
  int x, y, z;
  int xm, xp, ym, yp, zm, zp;  // periodic neighbours
};

__device__ __forceinline__ NodeCoord make_coord(int x, int y, int z, const Consts& k) {
  NodeCoord c;
  c.x = x; c.y = y; c.z = z;
  c.xm = (x == 0) ? k.nx - 1 : x - 1;
  c.xp = (x == k.nx - 1) ? 0 : x + 1;
  c.ym = (y == 0) ? k.ny - 1 : y - 1;
  c.yp = (y == k.ny - 1) ? 0 : y + 1;
  c.zm = (z == 0) ? k.nz - 1 : z - 1;
  c.zp = (z == k.nz - 1) ? 0 : z + 1;
  return c;
}

// Slot from which the node gathers f_a: (a, x - ebar_a) or, across a wall, (opp(a), x);
// in the AA layout between calls, (a, x).  64-bit element index (any state size).
// WX = false compiles the x-wall test away (for callers that know x is periodic).
template <int A, bool WX = true>
__device__ __forceinline__ int64_t gather_slot(const NodeCoord& c, const Consts& k) {
  constexpr int ex = kEx[A], ey = kEy[A], ez = kEz[A];
  constexpr int opp = opposite_of(A);
  if (k.aa) return slot_of<A>(c.x, c.y, c.z, k);  // natural order
  const int xs = ex == 0 ? c.x : (ex > 0 ? c.xm : c.xp);
  const int ys = ey == 0 ? c.y : (ey > 0 ? c.ym : c.yp);
  const int zs = ez == 0 ? c.z : (ez > 0 ? c.zm : c.zp);
  bool wall = false;
  if (WX && ex != 0) wall |= k.bb_x && (ex > 0 ? c.x == 0 : c.x == k.nx - 1);
  if (ey != 0) wall |= k.bb_y && (ey > 0 ? c.y == 0 : c.y == k.ny - 1);
  if (ez != 0) wall |= k.bb_z && (ez > 0 ? c.z == 0 : c.z == k.nz - 1);
  return wall ? slot_of<opp>(c.x, c.y, c.z, k) : slot_of<A>(xs, ys, zs, k);
}

// Slot that the next step gathers the node's own slot (B, x) from: (B, x + ebar_B), or,
// where x + ebar_B lies beyond a wall, the node's own (opp(B), x) (bounce-back).  In the
// adjoint arrays (gathered-population order) it holds the cotangent of (B, x).  64-bit
// element index; not for the AA layout.
template <int B, bool WX = true>
__device__ __forceinline__ int64_t downstream_slot(const NodeCoord& c, const Consts& k) {
  constexpr int ex = kEx[B], ey = kEy[B], ez = kEz[B];
  constexpr int opp = opposite_of(B);
  const int xs = ex == 0 ? c.x : (ex > 0 ? c.xp : c.xm);
  const int ys = ey == 0 ? c.y : (ey > 0 ? c.yp : c.ym);
  const int zs = ez == 0 ? c.z : (ez > 0 ? c.zp : c.zm);
  bool wall = false;
  if (WX && ex != 0) wall |= k.bb_x && (ex > 0 ? c.x == k.nx - 1 : c.x == 0);
  if (ey != 0) wall |= k.bb_y && (ey > 0 ? c.y == k.ny - 1 : c.y == 0);
  if (ez != 0) wall |= k.bb_z && (ez > 0 ? c.z == k.nz - 1 : c.z == 0);
  return wall ? slot_of<opp>(c.x, c.y, c.z, k) : slot_of<B>(xs, ys, zs, k);
}

template <int A, int ST, bool WX = true>
__device__ __forceinline__ float gather_dev(const typename Store<ST>::T* __restrict__ src,
                                            const NodeCoord& c, const Consts& k) {
  const float v = Store<ST>::load(src + gather_slot<A, WX>(c, k));
  return decode_scale<ST>(v, wclass(A), k);
}

template <int ST, int A = 0, bool WX = true>
__device__ __forceinline__ void gather_all(const typename Store<ST>::T* __restrict__ src,
                                           const NodeCoord& c, const Consts& k, float (&df)[27]) {
  df[A] = gather_dev<A, ST, WX>(src, c, k);
  if constexpr (A + 1 < 27) gather_all<ST, A + 1, WX>(src, c, k, df);
}

// ----------------------------------------------------------------- moments
// Raw moments of order <= 2 of the deviations, in cubic (ebar) units,
// factorised over z, then y, then x (App. A restricted to orders <= 2).
struct LowMoments {
  float m000, m100, m010, m001, m200, m020, m002, m110, m101, m011;
};

__device__ __forceinline__ LowMoments low_moments(const float (&df)[27]) {
  float Z0[3][3], Z1[3][3], Z2[3][3];
#pragma unroll
  for (int i = 0; i < 3; ++i)
#pragma unroll
    for (int j = 0; j < 3; ++j) {
      const float m = df[dir_of(i, j, 0)], o = df[dir_of(i, j, 1)], p = df[dir_of(i, j, 2)];
      Z2[i][j] = p + m;
      Z1[i][j] = p - m;
      Z0[i][j] = Z2[i][j] + o;
    }
  float Y00[3], Y10[3], Y20[3], Y01[3], Y11[3], Y02[3];
#pragma unroll
  for (int i = 0; i < 3; ++i) {
    Y20[i] = Z0[i][2] + Z0[i][0];
    Y10[i] = Z0[i][2] - Z0[i][0];
    Y00[i] = Y20[i] + Z0[i][1];
    Y11[i] = Z1[i][2] - Z1[i][0];
    Y01[i] = Z1[i][0] + Z1[i][1] + Z1[i][2];
    Y02[i] = Z2[i][0] + Z2[i][1] + Z2[i][2];
  }
  LowMoments M;
  M.m200 = Y00[2] + Y00[0];
  M.m100 = Y00[2] - Y00[0];
  M.m000 = M.m200 + Y00[1];
  M.m110 = Y10[2] - Y10[0];
  M.m010 = Y10[0] + Y10[1] + Y10[2];
  M.m020 = Y20[0] + Y20[1] + Y20[2];
  M.m101 = Y01[2] - Y01[0];
  M.m001 = Y01[0] + Y01[1] + Y01[2];
  M.m011 = Y11[0] + Y11[1] + Y11[2];
  M.m002 = Y02[0] + Y02[1] + Y02[2];
  return M;
}

// ----------------------------------------------------------------- per-axis vectors
// Along one axis (speed c, velocity u), entries for ebar = -1, 0, +1:
//   D  = E(u) - E(0): equilibrium weights minus rest weights
//   A0, A1, A2: populations of the unit central moments (1,0,0), (0,1,0),
//   (0,0,1) of that axis (the 1D inverse of the raw/central moment maps).
struct AxisVec {
  float W0[3], E[3], D[3], A0[3], A1[3], A2[3];
};

__device__ __forceinline__ AxisVec axis_vectors(float u, int d, const Consts& k) {
  AxisVec v;
  const float ic = k.ic[d], ic2 = k.ic2[d];
  const float q = u * u * ic2, h = u * ic;
  v.W0[0] = k.w0s[d]; v.W0[1] = k.w0c[d]; v.W0[2] = k.w0s[d];
  v.D[0] = 0.5f * (q - h); v.D[1] = -q; v.D[2] = 0.5f * (q + h);
  v.A0[0] = v.D[0]; v.A0[1] = 1.0f - q; v.A0[2] = v.D[2];
  const float uic2 = u * ic2, hic = 0.5f * ic;
  v.A1[0] = uic2 - hic; v.A1[1] = -2.0f * uic2; v.A1[2] = uic2 + hic;
  v.A2[0] = 0.5f * ic2; v.A2[1] = -ic2; v.A2[2] = 0.5f * ic2;
#pragma unroll
  for (int i = 0; i < 3; ++i) v.E[i] = v.W0[i] + v.D[i];
  return v;
}

// ----------------------------------------------------------------- collision
// Post-collision deviations of one node (the collide bullets of Sec. 3.2 with
// the App. D collision), for unit higher-order rate in the deviation form
//   f~ - w rho0 = d_rho E(x)E(x)E + rho0 [D(x)E(x)E + W0(x)D(x)E + W0(x)W0(x)D]
//                 + sum over the first/second-order non-equilibrium central
//                   moments Delta_mnp of Delta_mnp A_m(x)A_n(x)A_p,
// which equals P^-1 S^-1 F(-u) applied to the post-collision central moments.
// CORR: 0 none, 1 low-Mach theta, 2 theta with the 3u^2 terms, 3 as 2 plus the
// density-gradient terms (gx, gy, gz = grad rho, used only when CORR == 3).
// RAW: relax raw instead of central moments (the raw-moment scheme of Sec. 7).
// With unit higher-order rates the two schemes share every post-collision
// moment of order <= 2; the raw scheme sets the higher raw moments to their
// equilibria plus half the source, so its relaxed second-order
// non-equilibrium parts Delta map back through the per-axis basis at u = 0
// (A0 = (0, 1, 0), A1 = (-1, 0, 1)/(2c), A2 unchanged) instead of at u.
// HI: a general rate w of the moments of order >= 3 (k.omega_hi).  Those
// moments carry no source and all relax with w, so by the completeness of the
// 27 moments the collision becomes
//   f~ = w f_eq + (1 - w) f + (1 - w/2) s + sum_2 Delta'_mnp A_m(x)A_n(x)A_p,
// s the population of the central source F (first order only), with the
// second-order factors (1 - omega) replaced by (w - omega); the same holds in
// the raw scheme.  w = 1 gives the form above.
template <int CORR, bool RAW = false, bool HI = false>
__device__ __forceinline__ void collide_node(const float (&df)[27], float fx, float fy, float fz,
                                             const Consts& k, float (&out)[27],
                                             float grx = 0.0f, float gry = 0.0f, float grz = 0.0f) {
  const LowMoments M = low_moments(df);
  const float r = k.r, s = k.s, cs2 = k.cs2, rho0 = k.rho0;
  const float drho = M.m000;
  const float jx = M.m100, jy = r * M.m010, jz = s * M.m001;
  const float Pxx = M.m200, Pyy = k.c2[1] * M.m020, Pzz = k.c2[2] * M.m002;
  const float Pxy = r * M.m110, Pxz = s * M.m101, Pyz = (r * s) * M.m011;
  const float rho = rho0 + drho;
  // 1/rho: hardware reciprocal refined by one Newton step (about 1 ulp)
  float irho = __builtin_amdgcn_rcpf(rho);
  irho = irho * (2.0f - rho * irho);
  const float ux = (jx + 0.5f * fx) * irho;
  const float uy = (jy + 0.5f * fy) * irho;
  const float uz = (jz + 0.5f * fz) * irho;
  const float uxx = ux * ux, uyy = uy * uy, uzz = uz * uz;
  const float uF_x = ux * fx, uF_y = uy * fy, uF_z = uz * fz;

  // non-equilibrium parts of the combined second-order central moments (eq. 45-46, e_rho = 0)
  const float Rb = (Pxx + Pyy + Pzz) - 3.0f * cs2 * drho - rho * (uxx + uyy + uzz) + (uF_x + uF_y + uF_z);
  const float Rs1 = (Pxx - Pyy) - rho * (uxx - uyy) + (uF_x - uF_y);
  const float Rs2 = (Pxx - Pzz) - rho * (uxx - uzz) + (uF_x - uF_z);
  const float kxy = Pxy - rho * ux * uy + 0.5f * (ux * fy + uy * fx);
  const float kxz = Pxz - rho * ux * uz + 0.5f * (ux * fz + uz * fx);
  const float kyz = Pyz - rho * uy * uz + 0.5f * (uy * fz + uz * fy);

  const float wn = k.omega_nu, wx = k.omega_xi;
  float c2d1 = 0.0f, c2d2 = 0.0f, c2s = 0.0f;
  if constexpr (CORR != 0) {
    // strain-rate system of App. D divided by rho: C/rho . (rho du) = R
    const float g = (CORR >= 2) ? 1.5f : 0.0f;
    const float inw = 2.0f * cs2 / wn, inx = 2.0f * cs2 / wx;
    const float ax = 0.5f * (3.0f * cs2 - 1.0f), ay = 0.5f * (3.0f * cs2 - k.c2[1]), az = 0.5f * (3.0f * cs2 - k.c2[2]);
    const float csx = -inw + ax + g * uxx, cbx = -inx + ax + g * uxx;
    const float csy = inw - ay - g * uyy, cby = -inx + ay + g * uyy;
    const float csz = inw - az - g * uzz, cbz = -inx + az + g * uzz;
    const float det = -csx * csz * cby - csy * (csx * cbz - csz * cbx);
    // density-gradient terms e_sr1, e_sr2, e_br of App. D (A, B, C = a_d u_d);
    // zero without the full corrections, and then not added at all (x + 0 is
    // not folded by the compiler, as it turns -0 into +0)
    float es1 = 0.0f, es2 = 0.0f, eb = 0.0f;
    float Rs1e = Rs1, Rs2e = Rs2, Rbe = Rb;
    if constexpr (CORR == 3) {
      const float tA = ax * ux * grx, tB = ay * uy * gry, tC = az * uz * grz;
      es1 = tB - tA;
      es2 = tC - tA;
      eb = -(tA + tB + tC);
      Rs1e += es1;
      Rs2e += es2;
      Rbe += eb;
    }
    // closed-form solution of eq. 49 (the corrections only need a few digits of it)
    const float gx = (-csz * cby * Rs1e - csy * (cbz * Rs2e - csz * Rbe)) * __builtin_amdgcn_rcpf(det);
    const float gy = (Rs1e - csx * gx) * __builtin_amdgcn_rcpf(csy);
    const float gz = (Rs2e - csx * gx) * __builtin_amdgcn_rcpf(csz);
    // theta / rho of eq. 38-40 (App. D), times rho du
    const float hn = 1.0f / wn - 0.5f, hx = 1.0f / wx - 0.5f;
    const float g3 = (CORR >= 2) ? 3.0f : 0.0f;
    const float tx = -(g3 * uxx + 2.0f * ax), ty = -(g3 * uyy + 2.0f * ay), tz = -(g3 * uzz + 2.0f * az);
    // lambda . grad rho of eq. 38-40 equals 2 (1/omega - 1/2) times the e terms above
    float l1 = tx * gx - ty * gy, l2 = tx * gx - tz * gz, lb = tx * gx + ty * gy + tz * gz;
    if constexpr (CORR == 3) {
      l1 += 2.0f * es1;
      l2 += 2.0f * es2;
      lb += 2.0f * eb;
    }
    c2d1 = hn * l1;
    c2d2 = hn * l2;
    c2s = hx * lb;
  }
  // relaxation of the combined moments, then segregation (B^-1 of App. D)
  const float wh = HI ? k.omega_hi : 1.0f;
  const float D2s = (wh - wx) * Rb + wx * c2s;
  const float D2d1 = (wh - wn) * Rs1 + wn * c2d1;
  const float D2d2 = (wh - wn) * Rs2 + wn * c2d2;
  constexpr float third = 1.0f / 3.0f;
  const float Dxx = (D2s + D2d1 + D2d2) * third;
  const float Dyy = (D2s - 2.0f * D2d1 + D2d2) * third;
  const float Dzz = (D2s + D2d1 - 2.0f * D2d2) * third;
  const float Dxy = (wh - wn) * kxy, Dxz = (wh - wn) * kxz, Dyz = (wh - wn) * kyz;
  const float hF = 1.0f - 0.5f * wh;  // post-collision k_100 = F/2 (unit rate)
  const float Dx = hF * fx, Dy = hF * fy, Dz = hF * fz;
  const float drhoh = wh * drho, rho0h = wh * rho0;  // equilibrium part, times w

  const AxisVec X = axis_vectors(ux, 0, k);
  const AxisVec Y = axis_vectors(uy, 1, k);
  const AxisVec Z = axis_vectors(uz, 2, k);
  if constexpr (!RAW) {
#pragma unroll
    for (int i = 0; i < 3; ++i) {
      const float eE = drhoh * X.E[i] + rho0h * X.D[i];
      const float eW = rho0h * X.W0[i];
      const float a0 = Dx * X.A1[i] + Dxx * X.A2[i];
      const float a1 = Dy * X.A0[i] + Dxy * X.A1[i];
      const float a2 = Dyy * X.A0[i];
      const float b0 = Dz * X.A0[i] + Dxz * X.A1[i];
      const float b1 = Dyz * X.A0[i];
      const float c0 = Dzz * X.A0[i];
      // The per-axis vectors satisfy E = W0 + D, A0 = D at ebar = -1, +1 and
      // 1 + D at ebar = 0, and W0, A2 take equal values at -1 and +1.  Along y
      // and z the sums below use these identities; with QW = eW Y.W0 the z sums
      // are QE Z.E + QW Z.D + Q0 Z.A0 + Q1 Z.A1 + Q2 Z.A2, where
      // S = QE + QW + Q0 = (eE + eW) Y.E + Q0 multiplies Z.D.
      const float eEW = eE + eW;
      const float P = eE * Y.W0[0], R = a2 * Y.A2[0];
      const float QEs[3] = {P + eEW * Y.D[0], eE * Y.E[1] + eW * Y.D[1], P + eEW * Y.D[2]};
      const float Q0s[3] = {R + a0 * Y.D[0] + a1 * Y.A1[0], a0 * Y.A0[1] + a1 * Y.A1[1] + a2 * Y.A2[1],
                            R + a0 * Y.D[2] + a1 * Y.A1[2]};
#pragma unroll
      for (int j = 0; j < 3; ++j) {
        const float QE = QEs[j], Q0 = Q0s[j];
        const float Q1 = b0 * Y.A0[j] + b1 * Y.A1[j];
        const float Q2 = c0 * Y.A0[j];
        const float S = eEW * Y.E[j] + Q0;
        const float T = QE * Z.W0[0] + Q2 * Z.A2[0];
        out[dir_of(i, j, 0)] = T + S * Z.D[0] + Q1 * Z.A1[0];
        out[dir_of(i, j, 2)] = T + S * Z.D[2] + Q1 * Z.A1[2];
        out[dir_of(i, j, 1)] = QE * Z.W0[1] + Q0 + S * Z.D[1] + Q1 * Z.A1[1] + Q2 * Z.A2[1];
      }
    }
  } else {
    // equilibrium and first-order source through the basis at u, second order through the basis at 0
    const float hx = 0.5f * k.ic[0], hy = 0.5f * k.ic[1], hz = 0.5f * k.ic[2];
    const float cxy = Dxy * hx * hy, cxz = Dxz * hx * hz, cyz = Dyz * hy * hz;
#pragma unroll
    for (int i = 0; i < 3; ++i) {
      const float eE = drhoh * X.E[i] + rho0h * X.D[i];
      const float eW = rho0h * X.W0[i];
      const float a0 = Dx * X.A1[i];
      const float a1 = Dy * X.A0[i];
      const float b0 = Dz * X.A0[i];
#pragma unroll
      for (int j = 0; j < 3; ++j) {
        const float QE = eE * Y.E[j] + eW * Y.D[j];
        const float QW = eW * Y.W0[j];
        const float Q0 = a0 * Y.A0[j] + a1 * Y.A1[j];
        const float Q1 = b0 * Y.A0[j];
#pragma unroll
        for (int l = 0; l < 3; ++l) {
          float v = QE * Z.E[l] + QW * Z.D[l] + Q0 * Z.A0[l] + Q1 * Z.A1[l];
          // second-order Delta_mnp A_m(0) A_n(0) A_p(0): most products vanish at compile time
          if (j == 1 && l == 1) v += Dxx * X.A2[i];
          if (i == 1 && l == 1) v += Dyy * Y.A2[j];
          if (i == 1 && j == 1) v += Dzz * Z.A2[l];
          if (l == 1) v += cxy * (float)((i - 1) * (j - 1));
          if (j == 1) v += cxz * (float)((i - 1) * (l - 1));
          if (i == 1) v += cyz * (float)((j - 1) * (l - 1));
          out[dir_of(i, j, l)] = v;
        }
      }
    }
  }
  if constexpr (HI) {
    const float wl = 1.0f - wh;
#pragma unroll
    for (int a = 0; a < 27; ++a) out[a] += wl * df[a];
  }
}

// Values made opaque to the optimiser (no instruction is emitted).  Every
// forward kernel runs the collision between such fences, so the compiler
// fuses its multiply-adds the same way in each of them whatever code
// surrounds it, and the kernels that must agree bit for bit (two-buffer and
// AA steps, one and two nodes per thread) round identically.
template <int N>
__device__ __forceinline__ void fence_values(float (&v)[N]) {
#pragma unroll
  for (int i = 0; i < N; ++i) asm volatile("" : "+v"(v[i]));
}

__device__ __forceinline__ void fence_value(float& v) { asm volatile("" : "+v"(v)); }

// IN: fence the inputs too.  The 16-bit kernels with unit higher-order rate
// leave them open: their decode (an exact conversion and a power-of-two scale)
// folds into the first moment sums as mixed-precision multiply-adds, which
// round like separate operations because the product is exact.  With a general
// higher-order rate the inputs also enter the output ((1 - w) f), so they are
// fenced there.
template <int CORR, bool RAW = false, bool HI = false, bool IN = true>
__device__ __forceinline__ void collide_fenced(float (&df)[27], float fx, float fy, float fz, const Consts& k,
                                               float (&out)[27], float grx = 0.0f, float gry = 0.0f,
                                               float grz = 0.0f) {
  if constexpr (IN) {
    fence_values(df);
    fence_value(fx);
    fence_value(fy);
    fence_value(fz);
  }
  collide_node<CORR, RAW, HI>(df, fx, fy, fz, k, out, grx, gry, grz);
  fence_values(out);
}

// Momentum-augmented bounce-back (Sec. 4) applied where the populations are
// stored: the slot (alpha, x) of a population that leaves the fluid through a
// wall is read only by the bounce-back gather of node x itself, so the
// colliding node writes f~_alpha - [f_eq_alpha - f_eq_alphabar](rho, u_w)
// there, rho being its own density (the fluid density the paper assigns to
// the wall) and u_w the face velocity (an edge or corner link takes the mean
// over the moving faces it crosses, so a lid meets the side walls without a
// mass source).  f_eq is the product-form equilibrium; for a lid moving along
// x the bracket is the coefficient list of eq. 69.
__device__ __forceinline__ float weq1(int e, float u, int d, const Consts& k) {
  const float q = (k.cs2 + u * u) * k.ic2[d];
  return e == 0 ? 1.0f - q : 0.5f * q + 0.5f * (float)e * u * k.ic[d];
}

// Wall coefficient of the outgoing direction A at node (x, y, z):
// f_eq_A - f_eq_Abar per unit density at the link's wall velocity, or 0 when
// the link does not leave through a moving face.
template <int A>
__device__ __forceinline__ float moving_wall_coef(int x, int y, int z, const Consts& k) {
  constexpr int ex = kEx[A], ey = kEy[A], ez = kEz[A];
  int cnt = 0;
  float ux = 0.0f, uy = 0.0f, uz = 0.0f;
  auto cross = [&](int f) {
    if (!((k.moving >> f) & 1)) return;
    ++cnt;
    ux += k.wall_u[f][0];
    uy += k.wall_u[f][1];
    uz += k.wall_u[f][2];
  };
  if (ex != 0 && k.bb_x && (ex > 0 ? x == k.nx - 1 : x == 0)) cross(ex > 0 ? 1 : 0);
  if (ey != 0 && k.bb_y && (ey > 0 ? y == k.ny - 1 : y == 0)) cross(ey > 0 ? 3 : 2);
  if (ez != 0 && k.bb_z && (ez > 0 ? z == k.nz - 1 : z == 0)) cross(ez > 0 ? 5 : 4);
  if (cnt == 0) return 0.0f;
  const float inv = cnt == 1 ? 1.0f : (cnt == 2 ? 0.5f : 1.0f / 3.0f);
  ux *= inv; uy *= inv; uz *= inv;
  return weq1(ex, ux, 0, k) * weq1(ey, uy, 1, k) * weq1(ez, uz, 2, k)
       - weq1(-ex, ux, 0, k) * weq1(-ey, uy, 1, k) * weq1(-ez, uz, 2, k);
}

template <int A = 0>
__device__ __forceinline__ void moving_wall_terms(int x, int y, int z, float rho, const Consts& k, float (&out)[27]) {
  out[A] -= rho * moving_wall_coef<A>(x, y, z, k);
  if constexpr (A + 1 < 27) moving_wall_terms<A + 1>(x, y, z, rho, k, out);
}

// Transpose of moving_wall_terms: the wall terms are -rho d_A with rho the sum of
// the gathered populations, so every population's cotangent gains -sum_A lam_A d_A.
template <int A = 0>
__device__ __forceinline__ float moving_wall_vjp(int x, int y, int z, const Consts& k, const float (&lam)[27]) {
  const float c = lam[A] * moving_wall_coef<A>(x, y, z, k);
  if constexpr (A + 1 < 27) return c + moving_wall_vjp<A + 1>(x, y, z, k, lam);
  return c;
}

// Exact local conservation for FP32 storage.  In exact arithmetic the
// collision keeps the mass and adds F to the momentum; in FP32 the rounding
// of the 27 outputs leaves a residual of a few 1e-9 per node that repeats
// almost unchanged from step to step on a slowly varying flow and therefore
// accumulates.  The per-direction changes out - in are small, so their FP32
// rounding is tiny; their mass and momentum are summed in FP64 and the
// residual goes into the rest population (mass) and the three axis pairs
// f_{1,2}, f_{3,4}, f_{5,6} (momentum, antisymmetrically, so their mass and
// second moments are unchanged).
__device__ __forceinline__ void conserve(const float (&df)[27], float fx, float fy, float fz,
                                         const Consts& k, float (&out)[27]) {
  double dm = 0.0, dx = 0.0, dy = 0.0, dz = 0.0;
#pragma unroll
  for (int a = 0; a < 27; ++a) {
    const double d = (double)(out[a] - df[a]);
    dm += d;
    if (kEx[a] != 0) dx += kEx[a] * d;
    if (kEy[a] != 0) dy += kEy[a] * d;
    if (kEz[a] != 0) dz += kEz[a] * d;
  }
  // residuals in ebar units: the momentum change must be F / c_d along each axis
  const float rm = (float)(-dm);
  const float rx = (float)((double)fx - dx);
  const float ry = (float)((double)(fy * k.ic[1]) - dy);
  const float rz = (float)((double)(fz * k.ic[2]) - dz);
  out[0] += rm;
  out[1] += 0.5f * rx;
  out[2] -= 0.5f * rx;
  out[3] += 0.5f * ry;
  out[4] -= 0.5f * ry;
  out[5] += 0.5f * rz;
  out[6] -= 0.5f * rz;
}

// Density gradient of the full corrections (App. D: an isotropic second-order
// finite difference) from a field of density deviations:
//   grad rho (x) = (1/cs2) sum_a w_a e_a rho(x + ebar_a).
// With the product weights w_a = Wx Wy Wz it factorises over the 3 x 3
// transverse neighbourhood of each column x' in {x-1, x, x+1}:
//   T(x') = sum_jl Wy_j Wz_l rho(x', y+j-1, z+l-1)
//   U(x') = sum_l  Wz_l [rho(x', y+1, z+l-1) - rho(x', y-1, z+l-1)]
//   V(x') = sum_j  Wy_j [rho(x', y+j-1, z+1) - rho(x', y+j-1, z-1)]
//   d_x rho = (T(x+1) - T(x-1)) / 2
//   d_y rho = sum_i Wx_i U(x+i-1) / (2 r),   d_z rho = sum_i Wx_i V(x+i-1) / (2 s).
// Periodic axes wrap; across a bounce-back wall the neighbour is the
// boundary node itself (its mirror image).
struct ColumnSums {
  float T, U, V;
};

// Row pointers of the 3 x 3 transverse neighbourhood: [y offset][z offset] ->
// the density field's row (y', z'), a uniform 64-bit pointer (any field size).
struct TransverseRows {
  const float* row[3][3];
};

__device__ __forceinline__ TransverseRows transverse_rows(const float* __restrict__ drho, int y, int z,
                                                          const Consts& k) {
  int ys[3], zs[3];
  if (k.bb_y) {
    ys[0] = y == 0 ? 0 : y - 1; ys[2] = y == k.ny - 1 ? y : y + 1;
  } else {
    ys[0] = y == 0 ? k.ny - 1 : y - 1; ys[2] = y == k.ny - 1 ? 0 : y + 1;
  }
  if (k.bb_z) {
    zs[0] = z == 0 ? 0 : z - 1; zs[2] = z == k.nz - 1 ? z : z + 1;
  } else {
    zs[0] = z == 0 ? k.nz - 1 : z - 1; zs[2] = z == k.nz - 1 ? 0 : z + 1;
  }
  ys[1] = y;
  zs[1] = z;
  TransverseRows t;
#pragma unroll
  for (int j = 0; j < 3; ++j)
#pragma unroll
    for (int l = 0; l < 3; ++l) t.row[j][l] = drho + ((int64_t)zs[l] * k.ny + ys[j]) * k.nx;
  return t;
}

template <typename T>
__device__ __forceinline__ T ld_off(const T* __restrict__ base, uint32_t idx);

__device__ __forceinline__ ColumnSums column_sums(const TransverseRows& t, int xc, const Consts& k) {
  float v[3][3];
#pragma unroll
  for (int j = 0; j < 3; ++j)
#pragma unroll
    for (int l = 0; l < 3; ++l) v[j][l] = ld_off(t.row[j][l], (uint32_t)xc);
  const float wy[3] = {k.w0s[1], k.w0c[1], k.w0s[1]};
  const float wz[3] = {k.w0s[2], k.w0c[2], k.w0s[2]};
  // -0 is the exact additive identity, so the first product needs no add
  ColumnSums c{-0.0f, -0.0f, -0.0f};
#pragma unroll
  for (int a = 0; a < 3; ++a) {
    c.U += wz[a] * (v[2][a] - v[0][a]);
    c.V += wy[a] * (v[a][2] - v[a][0]);
#pragma unroll
    for (int b = 0; b < 3; ++b) c.T += wy[a] * wz[b] * v[a][b];
  }
  return c;
}

// Block-cooperative gradient for the nodes of one row segment (blockDim.x
// consecutive x, one y, z): each thread reduces its own column, two threads
// reduce the halo columns x0 - 1 and x_last + 1 (wrapped or mirrored), the x
// neighbours are exchanged through LDS.  Every thread of the block must call
// it (it contains a barrier); threads with x >= nx pass active = false.
__device__ __forceinline__ void density_gradient_block(const float* __restrict__ drho, int x, int y, int z,
                                                       bool active, const Consts& k, float (&lds)[3][258],
                                                       float& gx, float& gy, float& gz) {
  const int t = (int)threadIdx.x;
  const TransverseRows rows = transverse_rows(drho, y, z, k);
  if (active) {
    const ColumnSums c = column_sums(rows, x, k);
    lds[0][t + 1] = c.T; lds[1][t + 1] = c.U; lds[2][t + 1] = c.V;
    if (t == 0) {
      const ColumnSums h = column_sums(rows, x == 0 ? (k.bb_x ? 0 : k.nx - 1) : x - 1, k);
      lds[0][0] = h.T; lds[1][0] = h.U; lds[2][0] = h.V;
    }
    if (t == (int)blockDim.x - 1 || x == k.nx - 1) {
      const ColumnSums h = column_sums(rows, x == k.nx - 1 ? (k.bb_x ? x : 0) : x + 1, k);
      lds[0][t + 2] = h.T; lds[1][t + 2] = h.U; lds[2][t + 2] = h.V;
    }
  }
  __syncthreads();
  if (active) {
    const float wc = k.w0c[0], ws = k.w0s[0];
    gx = 0.5f * (lds[0][t + 2] - lds[0][t]);
    gy = 0.5f * k.ic[1] * (ws * lds[1][t] + wc * lds[1][t + 1] + ws * lds[1][t + 2]);
    gz = 0.5f * k.ic[2] * (ws * lds[2][t] + wc * lds[2][t + 1] + ws * lds[2][t + 2]);
  }
}

// The same gradient for two nodes per thread (nodes x0 = 2t and x0 + 1 of a row
// segment of 2 blockDim.x nodes): each thread reduces its two columns, the first
// and last thread the halo columns, and the neighbours come from LDS
// (lds[c][2 blockDim.x + 2]).  The per-node arithmetic is that of
// density_gradient_block.  Every thread of the block must call it.
__device__ __forceinline__ void density_gradient_pair_block(const float* __restrict__ drho, int x0, int y, int z,
                                                            bool active, const Consts& k, float (&lds)[3][258],
                                                            float (&g)[2][3]) {
  const int t = (int)threadIdx.x;
  const TransverseRows rows = transverse_rows(drho, y, z, k);
  if (active) {
    const ColumnSums c0 = column_sums(rows, x0, k), c1 = column_sums(rows, x0 + 1, k);
    lds[0][2 * t + 1] = c0.T; lds[1][2 * t + 1] = c0.U; lds[2][2 * t + 1] = c0.V;
    lds[0][2 * t + 2] = c1.T; lds[1][2 * t + 2] = c1.U; lds[2][2 * t + 2] = c1.V;
    if (t == 0) {
      const ColumnSums h = column_sums(rows, x0 == 0 ? (k.bb_x ? 0 : k.nx - 1) : x0 - 1, k);
      lds[0][0] = h.T; lds[1][0] = h.U; lds[2][0] = h.V;
    }
    if (t == (int)blockDim.x - 1 || x0 + 1 == k.nx - 1) {
      const ColumnSums h = column_sums(rows, x0 + 1 == k.nx - 1 ? (k.bb_x ? x0 + 1 : 0) : x0 + 2, k);
      lds[0][2 * t + 3] = h.T; lds[1][2 * t + 3] = h.U; lds[2][2 * t + 3] = h.V;
    }
  }
  __syncthreads();
  if (active) {
    const float wc = k.w0c[0], ws = k.w0s[0];
#pragma unroll
    for (int h = 0; h < 2; ++h) {
      const int i = 2 * t + h;  // the node's left neighbour column in LDS
      g[h][0] = 0.5f * (lds[0][i + 2] - lds[0][i]);
      g[h][1] = 0.5f * k.ic[1] * (ws * lds[1][i] + wc * lds[1][i + 1] + ws * lds[1][i + 2]);
      g[h][2] = 0.5f * k.ic[2] * (ws * lds[2][i] + wc * lds[2][i + 1] + ws * lds[2][i + 2]);
    }
  }
}

// Grid row (y, z) of row number `rowid`: y fastest, or in tiles of ty rows in y,
// z-major inside a tile (the rows that read one upstream row then run close in time).
__device__ __forceinline__ void tiled_row(uint32_t rowid, uint32_t ty, const Consts& k, int& y, int& z) {
  if (ty <= 1) {
    y = (int)(rowid % (uint32_t)k.ny);
    z = (int)(rowid / (uint32_t)k.ny);
  } else {
    const uint32_t per_tile = ty * (uint32_t)k.nz;
    const uint32_t tile = rowid / per_tile, rem = rowid % per_tile;
    z = (int)(rem / ty);
    y = (int)(tile * ty + rem % ty);
  }
}

// XCD-aware block order: hardware hands consecutive workgroups to the 8 XCDs
// in turn; renumber so that each XCD walks one contiguous range of tiles
// (neighbouring rows share cache lines through that XCD's L2).
__device__ __forceinline__ uint32_t xcd_block(uint32_t b, uint32_t nb) {
  constexpr uint32_t X = 8;
  const uint32_t per = nb / X, rem = nb % X;
  const uint32_t xcd = b % X, i = b / X;
  return xcd < rem ? xcd * (per + 1) + i : rem * (per + 1) + (xcd - rem) * per + i;
}

// Load/store through a uniform base pointer and a 32-bit element index (the
// byte offset fits in 32 bits), so the address is SGPR base + VGPR offset.
template <typename T>
__device__ __forceinline__ T ld_off(const T* __restrict__ base, uint32_t idx) {
  return *reinterpret_cast<const T*>(reinterpret_cast<const char*>(base) + (uint32_t)(idx * (uint32_t)sizeof(T)));
}

// Non-temporal variant of ld_off, for population lines that no other wave reads
// in the same step.
template <typename T>
__device__ __forceinline__ T ld_off_nt(const T* __restrict__ base, uint32_t idx) {
  const T* p = reinterpret_cast<const T*>(reinterpret_cast<const char*>(base) + (uint32_t)(idx * (uint32_t)sizeof(T)));
  if constexpr (sizeof(T) == 4) {
    return __builtin_bit_cast(T, __builtin_nontemporal_load(reinterpret_cast<const float*>(p)));
  } else {
    return __builtin_bit_cast(T, __builtin_nontemporal_load(reinterpret_cast<const unsigned short*>(p)));
  }
}

template <bool NT, typename T>
__device__ __forceinline__ T ld_pop(const T* __restrict__ base, uint32_t idx) {
  if constexpr (NT) return ld_off_nt(base, idx);
  else return ld_off(base, idx);
}

// The same 32-bit value, defined anew where it is called.  A node offset that
// the loads already used reaches the stores of another basic block widened to
// 64 bits, and each store then adds its base in a 64-bit VALU operation; an
// offset defined next to the stores lets them take their base from SGPRs.
__device__ __forceinline__ uint32_t store_offset(uint32_t v) {
  asm volatile("" : "+v"(v));
  return v;
}

template <typename T>
__device__ __forceinline__ void st_off(T* __restrict__ base, uint32_t idx, T v) {
  *reinterpret_cast<T*>(reinterpret_cast<char*>(base) + (uint32_t)(idx * (uint32_t)sizeof(T))) = v;
}

template <typename T>
__device__ __forceinline__ void st_off_nt(T* __restrict__ base, uint32_t idx, T v) {
  T* p = reinterpret_cast<T*>(reinterpret_cast<char*>(base) + (uint32_t)(idx * (uint32_t)sizeof(T)));
  if constexpr (sizeof(T) == 4) {
    __builtin_nontemporal_store(__builtin_bit_cast(float, v), reinterpret_cast<float*>(p));
  } else {
    __builtin_nontemporal_store(__builtin_bit_cast(unsigned short, v), reinterpret_cast<unsigned short*>(p));
  }
}

// Upstream rows and x offsets of a node, for the row-addressed paths.
// row[j][l]: first element of the grid row (y - (j - 1), z - (l - 1)), the row a
// direction with ebar_y = j - 1, ebar_z = l - 1 pulls from (wrapped; on a wall
// axis the wrapped row is never used, the wall test selects the node's own
// slot instead).  The rows depend on y and z only, so they are uniform across
// a block and live in scalar registers: every access is a 64-bit scalar row
// address plus a small per-lane offset.  xo[i]: offset within a row of
// x - (i - 1) (wrapped).
struct Upstream {
  int64_t row[3][3];
  uint32_t xo[3];
};

__device__ __forceinline__ void upstream(int x, int y, int z, const Consts& k, Upstream& u) {
  u.xo[0] = xoff((uint32_t)(x == k.nx - 1 ? 0 : x + 1));
  u.xo[1] = xoff((uint32_t)x);
  u.xo[2] = xoff((uint32_t)(x == 0 ? k.nx - 1 : x - 1));
  const int ys[3] = {y == k.ny - 1 ? 0 : y + 1, y, y == 0 ? k.ny - 1 : y - 1};
  const int zs[3] = {z == k.nz - 1 ? 0 : z + 1, z, z == 0 ? k.nz - 1 : z - 1};
#pragma unroll
  for (int j = 0; j < 3; ++j)
#pragma unroll
    for (int l = 0; l < 3; ++l) u.row[j][l] = row_start(ys[j], zs[l], k);
}

// Global (address space 1) pointers.
template <typename T>
using global_t = __attribute__((address_space(1))) T;

// Uniform pointer pinned in scalar registers, as a global pointer.  Without the
// pin the compiler folds a chunk offset beyond the 4 KiB immediate range into
// per-lane 64-bit address arithmetic; with it every access is a scalar base
// plus a 32-bit lane offset plus an immediate (the position of the chunk within
// its group).  Only for pointers that are uniform across the wave.
template <typename T>
__device__ __forceinline__ global_t<T>* sgpr_ptr(T* p) {
  uint64_t v = reinterpret_cast<uint64_t>(p);
  asm volatile("" : "+s"(v));
  return reinterpret_cast<global_t<T>*>(v);
}

// Accesses through global pointers move the raw bits (a 16-bit type such as
// __half cannot be copied through an address-space-qualified reference).
template <typename T>
using raw_t = typename std::conditional<sizeof(T) == 4, uint32_t, unsigned short>::type;

template <typename T>
__device__ __forceinline__ const global_t<raw_t<T>>* raw_at(const global_t<T>* base, uint32_t idx) {
  return reinterpret_cast<const global_t<raw_t<T>>*>(reinterpret_cast<const global_t<char>*>(base) +
                                                     (uint32_t)(idx * (uint32_t)sizeof(T)));
}

template <typename T>
__device__ __forceinline__ global_t<raw_t<T>>* raw_at(global_t<T>* base, uint32_t idx) {
  return reinterpret_cast<global_t<raw_t<T>>*>(reinterpret_cast<global_t<char>*>(base) +
                                               (uint32_t)(idx * (uint32_t)sizeof(T)));
}

template <typename T>
__device__ __forceinline__ T ld_off(const global_t<T>* __restrict__ base, uint32_t idx) {
  return __builtin_bit_cast(T, *raw_at(base, idx));
}

template <typename T>
__device__ __forceinline__ T ld_off_nt(const global_t<T>* __restrict__ base, uint32_t idx) {
  return __builtin_bit_cast(T, __builtin_nontemporal_load(raw_at(base, idx)));
}

template <bool NT, typename T>
__device__ __forceinline__ T ld_pop(const global_t<T>* __restrict__ base, uint32_t idx) {
  if constexpr (NT) return ld_off_nt(base, idx);
  else return ld_off(base, idx);
}

template <typename T>
__device__ __forceinline__ void st_off(global_t<T>* __restrict__ base, uint32_t idx, T v) {
  *raw_at(base, idx) = __builtin_bit_cast(raw_t<T>, v);
}

template <typename T>
__device__ __forceinline__ void st_off_nt(global_t<T>* __restrict__ base, uint32_t idx, T v) {
  __builtin_nontemporal_store(__builtin_bit_cast(raw_t<T>, v), raw_at(base, idx));
}

// Chunk group of a direction: the three directions with the same (ebar_y,
// ebar_z), stored side by side (chunk_of(a) = 3 group_of(a) + ebar_x + 1).
constexpr int group_of(int a) { return group_index(kEy[a], kEz[a]); }

// Scalar bases of the nine chunk groups: pull[g] = group g of the row that its
// directions pull from (row[g / 3][g % 3]), own[g] = group g of the node's own row.
template <typename T>
struct GroupBases {
  global_t<T>* g[9];
};

template <typename T>
__device__ __forceinline__ GroupBases<T> pull_groups(T* state, const Upstream& u) {
  GroupBases<T> b;
#pragma unroll
  for (int g = 0; g < 9; ++g) b.g[g] = sgpr_ptr(state + u.row[group_ey(g) + 1][group_ez(g) + 1] + 3 * g * kB);
  return b;
}

template <typename T>
__device__ __forceinline__ GroupBases<T> own_groups(T* state, const Upstream& u) {
  GroupBases<T> b;
#pragma unroll
  for (int g = 0; g < 9; ++g) b.g[g] = sgpr_ptr(state + u.row[1][1] + 3 * g * kB);
  return b;
}

// AA odd step: odd[g] = group 8 - g (the opposite directions) of the row that
// group g pulls from.  Direction A (group g) reads its opposite's chunk there,
// at odd[g] + (1 - ebar_x) kB, and writes its own chunk in the row it pushes
// to, which is odd[8 - g] + (ebar_x + 1) kB.
template <typename T>
__device__ __forceinline__ GroupBases<T> aa_odd_groups(T* state, const Upstream& u) {
  GroupBases<T> b;
#pragma unroll
  for (int g = 0; g < 9; ++g) b.g[g] = sgpr_ptr(state + u.row[group_ey(g) + 1][group_ez(g) + 1] + 3 * (8 - g) * kB);
  return b;
}

// Slot array of direction A through its group's base (chunk position ebar_x + 1).
template <int A, typename T>
__device__ __forceinline__ global_t<T>* chunk_ptr(const GroupBases<T>& b) {
  return b.g[group_of(A)] + (kEx[A] + 1) * kB;
}

// A copy of the x offsets defined anew for a block of stores (store_offset).
__device__ __forceinline__ Upstream store_upstream(const Upstream& u) {
  Upstream s = u;
#pragma unroll
  for (int i = 0; i < 3; ++i) s.xo[i] = store_offset(u.xo[i]);
  return s;
}

// Element of the chunk row that direction A pulls from: add xo[ebar_x + 1].
template <int A>
__device__ __forceinline__ int64_t pull_row(const Upstream& u) {
  return u.row[kEy[A] + 1][kEz[A] + 1] + chunk_of(A) * kB;
}

// Walls with 32-bit offsets (the whole state below 4 GiB): the slot of f_A is
// (A, x - ebar_A) or, across a wall, (opp(A), x), as one 32-bit element offset
// from the start of the state; a wall costs a compare and a select.
struct WallFlags {
  bool lx, hx, ly, hy, lz, hz;  // upstream node beyond the wall at the low / high end of an axis
};

__device__ __forceinline__ WallFlags wall_flags(int x, int y, int z, const Consts& k) {
  WallFlags w;
  w.lx = k.bb_x && x == 0;
  w.hx = k.bb_x && x == k.nx - 1;
  w.ly = k.bb_y && y == 0;
  w.hy = k.bb_y && y == k.ny - 1;
  w.lz = k.bb_z && z == 0;
  w.hz = k.bb_z && z == k.nz - 1;
  return w;
}

// Whether direction A's upstream node lies beyond a wall.
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

// 32-bit element of the node's own slot (A, x).
template <int A>
__device__ __forceinline__ uint32_t own_slot32(const Upstream& u) {
  return (uint32_t)u.row[1][1] + (uint32_t)(chunk_of(A) * kB) + u.xo[1];
}

// 32-bit element of slot (C, x - ebar_A): direction A's upstream node, chunk of C.
template <int A, int C>
__device__ __forceinline__ uint32_t upstream_slot32(const Upstream& u) {
  return (uint32_t)u.row[kEy[A] + 1][kEz[A] + 1] + (uint32_t)(chunk_of(C) * kB) + u.xo[kEx[A] + 1];
}

template <int A>
__device__ __forceinline__ uint32_t wall_slot32(const Upstream& u, const WallFlags& w) {
  return pulls_through_wall<A>(w) ? own_slot32<opposite_of(A)>(u) : upstream_slot32<A, A>(u);
}

// 32-bit form of downstream_slot: (B, x + ebar_B), or the own (opp(B), x) where
// x + ebar_B lies beyond a wall (exactly where opp(B) pulls through one).
template <int B>
__device__ __forceinline__ uint32_t downstream_slot32(const Upstream& u, const WallFlags& w) {
  constexpr int O = opposite_of(B);
  return pulls_through_wall<O>(w) ? own_slot32<O>(u) : upstream_slot32<O, B>(u);
}

// NT: 0 plain loads; 1 non-temporal loads; 2 non-temporal loads for the
// directions with ebar_x = 0 only.  A wave reads whole aligned lines for those;
// the x-shifted directions straddle a line that the neighbouring wave reads
// too, which plain loads keep in L2.
template <int NT>
constexpr bool nt_dir(int a) {
  return NT == 1 || (NT == 2 && kEx[a] == 0);
}

template <int ST, int NT = 0, int A = 0>
__device__ __forceinline__ void gather_walls32(const typename Store<ST>::T* __restrict__ base, const Upstream& u,
                                               const WallFlags& w, const Consts& k, float (&df)[27]) {
  const float v = Store<ST>::load_val(ld_pop<nt_dir<NT>(A)>(base, wall_slot32<A>(u, w)));
  df[A] = decode_scale<ST>(v, wclass(A), k);
  if constexpr (A + 1 < 27) gather_walls32<ST, NT, A + 1>(base, u, w, k, df);
}

template <int ST, int NT = 0, int I = 0>
__device__ __forceinline__ void gather_periodic(const GroupBases<const typename Store<ST>::T>& b, const Upstream& u,
                                                const Consts& k, float (&df)[27]) {
  constexpr int A = issue_dir(I);
  const float v = Store<ST>::load_val(ld_pop<nt_dir<NT>(A)>(chunk_ptr<A>(b), u.xo[kEx[A] + 1]));
  df[A] = decode_scale<ST>(v, wclass(A), k);
  if constexpr (I + 1 < 27) gather_periodic<ST, NT, I + 1>(b, u, k, df);
}

}  // namespace clbm
