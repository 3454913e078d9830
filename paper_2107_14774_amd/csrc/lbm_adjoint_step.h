// Reverse mode of the fused step (see the note below), templated on the storage
// type; each storage type is instantiated in lbm_adjoint_step_<type>.hip
// through AdjointKernels<ST>.
//
// The step maps the state h(t) to h(t+1) = C(S(h(t)); F) where S is the
// streaming permutation of slots and C the per-node collision.  The adjoint
// step gathers the node's populations from h(t) (as the forward did),
// recomputes the collision and applies the transpose of its Jacobian to the
// cotangents of the node's outputs, lambda(t+1); the result belongs to the
// slots the node gathered from.  S is a permutation, so with the adjoint
// arrays in gathered-population order (below) every element of lambda(t) is
// written exactly once, at the node's own slots, and no atomics are needed.
// The transpose is derived by hand from the factorised collision of
// lbm_device.h; along each axis the vectors satisfy dE/du = dD/du = dA0/du =
// A1 and dA1/du = 2 A2, which keeps the velocity derivatives short.
#pragma once

#include "lbm_internal.h"

// Occupancy requested from the register allocator for the adjoint step:
// 3 waves per SIMD fit the 16-bit variants without spills (measured faster
// on 384x384x192); the FP32 variants and those with a general higher-order
// rate would spill, so they get no bound.
#ifndef LBM_ADJ_WAVES_16
#define LBM_ADJ_WAVES_16 3
#endif
#ifndef LBM_ADJ_WAVES_32
#define LBM_ADJ_WAVES_32 1
#endif

namespace clbm {

// lambda^T dC/d(df, F) at one node: mu = (dC/d df)^T lam, gf = (dC/dF)^T lam.
// RAW: the raw-moment scheme, whose relaxed second-order non-equilibrium parts
// map back through the per-axis basis at u = 0 (collide_node): those terms
// carry no velocity dependence and their cotangents come from lam directly.
// HI: general higher-order rate w (collide_node): the equilibrium part scales
// by w, the source and second-order factors change, and mu gains (1 - w) lam.
// CORR 3 (full corrections): grx, gry, grz is the node's density gradient, and
// bgrad receives lam^T dC/d(grad rho) (the cotangent of the gradient).
template <int CORR, bool RAW = false, bool HI = false>
__device__ __forceinline__ void collide_vjp(const float (&df)[27], float fx, float fy, float fz, const Consts& k,
                                            const float (&lam)[27], float (&mu)[27], float& gfx, float& gfy,
                                            float& gfz, float grx = 0.0f, float gry = 0.0f, float grz = 0.0f,
                                            float* bgrad = nullptr) {
  // ---------------------------------------------------------------- forward recomputation
  const LowMoments M = low_moments(df);
  const float r = k.r, s = k.s, cs2 = k.cs2, rho0 = k.rho0;
  const float drho = M.m000;
  const float jx = M.m100, jy = r * M.m010, jz = s * M.m001;
  const float Pxx = M.m200, Pyy = k.c2[1] * M.m020, Pzz = k.c2[2] * M.m002;
  const float Pxy = r * M.m110, Pxz = s * M.m101, Pyz = (r * s) * M.m011;
  const float rho = rho0 + drho;
  float irho = __builtin_amdgcn_rcpf(rho);
  irho = irho * (2.0f - rho * irho);
  const float ux = (jx + 0.5f * fx) * irho, uy = (jy + 0.5f * fy) * irho, uz = (jz + 0.5f * fz) * irho;
  const float uxx = ux * ux, uyy = uy * uy, uzz = uz * uz;
  const float Rb = (Pxx + Pyy + Pzz) - 3.0f * cs2 * drho - rho * (uxx + uyy + uzz) + (ux * fx + uy * fy + uz * fz);
  const float Rs1 = (Pxx - Pyy) - rho * (uxx - uyy) + (ux * fx - uy * fy);
  const float Rs2 = (Pxx - Pzz) - rho * (uxx - uzz) + (ux * fx - uz * fz);
  const float kxy = Pxy - rho * ux * uy + 0.5f * (ux * fy + uy * fx);
  const float kxz = Pxz - rho * ux * uz + 0.5f * (ux * fz + uz * fx);
  const float kyz = Pyz - rho * uy * uz + 0.5f * (uy * fz + uz * fy);
  const float wn = k.omega_nu, wx = k.omega_xi;
  const float g = (CORR >= 2) ? 1.5f : 0.0f, g3 = 2.0f * g;
  const float hn = 1.0f / wn - 0.5f, hx = 1.0f / wx - 0.5f;
  float csx = 0, cbx = 0, csy = 1, cby = 0, csz = 1, cbz = 0, det = 1, gx = 0, gy = 0, gz = 0, tx = 0, ty = 0, tz = 0;
  float c2d1 = 0.0f, c2d2 = 0.0f, c2s = 0.0f;
  // the solve's right-hand sides: Rs1, Rs2, Rb plus the density-gradient terms e_sr1,
  // e_sr2, e_br of App. D with the full corrections (as in collide_node)
  float Rs1e = Rs1, Rs2e = Rs2, Rbe = Rb, es1 = 0.0f, es2 = 0.0f, eb = 0.0f;
  const float ax = 0.5f * (3.0f * cs2 - 1.0f), ay = 0.5f * (3.0f * cs2 - k.c2[1]), az = 0.5f * (3.0f * cs2 - k.c2[2]);
  if constexpr (CORR != 0) {
    const float inw = 2.0f * cs2 / wn, inx = 2.0f * cs2 / wx;
    csx = -inw + ax + g * uxx; cbx = -inx + ax + g * uxx;
    csy = inw - ay - g * uyy; cby = -inx + ay + g * uyy;
    csz = inw - az - g * uzz; cbz = -inx + az + g * uzz;
    det = -csx * csz * cby - csy * (csx * cbz - csz * cbx);
    if constexpr (CORR == 3) {
      const float tA = ax * ux * grx, tB = ay * uy * gry, tC = az * uz * grz;
      es1 = tB - tA;
      es2 = tC - tA;
      eb = -(tA + tB + tC);
      Rs1e += es1;
      Rs2e += es2;
      Rbe += eb;
    }
    gx = (-csz * cby * Rs1e - csy * (cbz * Rs2e - csz * Rbe)) * __builtin_amdgcn_rcpf(det);
    gy = (Rs1e - csx * gx) * __builtin_amdgcn_rcpf(csy);
    gz = (Rs2e - csx * gx) * __builtin_amdgcn_rcpf(csz);
    tx = -(g3 * uxx + 2.0f * ax); ty = -(g3 * uyy + 2.0f * ay); tz = -(g3 * uzz + 2.0f * az);
    // the lambda terms equal twice the e terms (collide_node)
    c2d1 = hn * (tx * gx - ty * gy + 2.0f * es1);
    c2d2 = hn * (tx * gx - tz * gz + 2.0f * es2);
    c2s = hx * (tx * gx + ty * gy + tz * gz + 2.0f * eb);
  }
  const float wh = HI ? k.omega_hi : 1.0f;
  const float D2s = (wh - wx) * Rb + wx * c2s;
  const float D2d1 = (wh - wn) * Rs1 + wn * c2d1;
  const float D2d2 = (wh - wn) * Rs2 + wn * c2d2;
  constexpr float third = 1.0f / 3.0f;
  const float Dxx = (D2s + D2d1 + D2d2) * third;
  const float Dyy = (D2s - 2.0f * D2d1 + D2d2) * third;
  const float Dzz = (D2s + D2d1 - 2.0f * D2d2) * third;
  const float Dxy = (wh - wn) * kxy, Dxz = (wh - wn) * kxz, Dyz = (wh - wn) * kyz;
  const float hF = 1.0f - 0.5f * wh;
  const float Dx = hF * fx, Dy = hF * fy, Dz = hF * fz;
  const float drhoh = wh * drho, rho0h = wh * rho0, rhoh = wh * rho;
  const AxisVec X = axis_vectors(ux, 0, k);
  const AxisVec Y = axis_vectors(uy, 1, k);
  const AxisVec Z = axis_vectors(uz, 2, k);

  // ---------------------------------------------------------------- reverse: output tensor products
  float bux = 0.0f, buy = 0.0f, buz = 0.0f, bdrho = 0.0f;
  float bDx = 0.0f, bDy = 0.0f, bDz = 0.0f, bDxx = 0.0f, bDyy = 0.0f, bDzz = 0.0f, bDxy = 0.0f, bDxz = 0.0f, bDyz = 0.0f;
  // second-order parts inside the basis at u (central scheme only)
  const float Exx = RAW ? 0.0f : Dxx, Eyy = RAW ? 0.0f : Dyy, Ezz = RAW ? 0.0f : Dzz;
  const float Exy = RAW ? 0.0f : Dxy, Exz = RAW ? 0.0f : Dxz, Eyz = RAW ? 0.0f : Dyz;
#pragma unroll
  for (int i = 0; i < 3; ++i) {
    const float eE = drhoh * X.E[i] + rho0h * X.D[i];
    const float eW = rho0h * X.W0[i];
    const float a0 = Dx * X.A1[i] + Exx * X.A2[i];
    const float a1 = Dy * X.A0[i] + Exy * X.A1[i];
    const float a2 = Eyy * X.A0[i];
    const float b0 = Dz * X.A0[i] + Exz * X.A1[i];
    const float b1 = Eyz * X.A0[i];
    const float c0 = Ezz * X.A0[i];
    float eEb = 0.0f, a0b = 0.0f, a1b = 0.0f, a2b = 0.0f, b0b = 0.0f, b1b = 0.0f, c0b = 0.0f;
#pragma unroll
    for (int j = 0; j < 3; ++j) {
      float LE = 0.0f, L0 = 0.0f, L1 = 0.0f, L2 = 0.0f;
#pragma unroll
      for (int l = 0; l < 3; ++l) {
        const float lv = lam[dir_of(i, j, l)];
        LE += lv * Z.E[l];
        L0 += lv * Z.A0[l];
        L1 += lv * Z.A1[l];
        L2 += lv * Z.A2[l];
      }
      const float QE = eE * Y.E[j] + eW * Y.D[j];
      const float QW = eW * Y.W0[j];
      const float Q0 = a0 * Y.A0[j] + a1 * Y.A1[j] + a2 * Y.A2[j];
      const float Q1 = b0 * Y.A0[j] + b1 * Y.A1[j];
      // d/du_z: E', D', A0' = A1 and A1' = 2 A2 (the cotangent of QW is not needed: QW is constant)
      buz += (QE + QW + Q0) * L1 + 2.0f * Q1 * L2;
      // y-vectors
      eEb += LE * Y.E[j];
      buy += LE * (eE + eW) * Y.A1[j];
      a0b += L0 * Y.A0[j];
      a1b += L0 * Y.A1[j];
      a2b += L0 * Y.A2[j];
      buy += L0 * (a0 * Y.A1[j] + 2.0f * a1 * Y.A2[j]);
      b0b += L1 * Y.A0[j];
      b1b += L1 * Y.A1[j];
      buy += L1 * (b0 * Y.A1[j] + 2.0f * b1 * Y.A2[j]);
      c0b += L2 * Y.A0[j];
      buy += L2 * c0 * Y.A1[j];
    }
    // x-coefficients
    bdrho += wh * eEb * X.E[i];
    bux += eEb * rhoh * X.A1[i];
    bDx += a0b * X.A1[i];
    bux += 2.0f * a0b * Dx * X.A2[i];
    bDy += a1b * X.A0[i];
    bux += a1b * Dy * X.A1[i];
    bDz += b0b * X.A0[i];
    bux += b0b * Dz * X.A1[i];
    if constexpr (!RAW) {
      bDxx += a0b * X.A2[i];
      bDxy += a1b * X.A1[i];
      bux += a1b * 2.0f * Dxy * X.A2[i];
      bDyy += a2b * X.A0[i];
      bux += a2b * Dyy * X.A1[i];
      bDxz += b0b * X.A1[i];
      bux += b0b * 2.0f * Dxz * X.A2[i];
      bDyz += b1b * X.A0[i];
      bux += b1b * Dyz * X.A1[i];
      bDzz += c0b * X.A0[i];
      bux += c0b * Dzz * X.A1[i];
    }
  }
  if constexpr (RAW) {
    // second-order parts through the basis at u = 0: A0 = e_1, A1 = (-1, 0, 1)/(2c), A2 as at u
    const float hx2 = 0.5f * k.ic[0], hy2 = 0.5f * k.ic[1], hz2 = 0.5f * k.ic[2];
#pragma unroll
    for (int i = 0; i < 3; ++i) {
      bDxx += lam[dir_of(i, 1, 1)] * X.A2[i];
      bDyy += lam[dir_of(1, i, 1)] * Y.A2[i];
      bDzz += lam[dir_of(1, 1, i)] * Z.A2[i];
#pragma unroll
      for (int j = 0; j < 3; ++j) {
        const float sgn = (float)((i - 1) * (j - 1));
        bDxy += sgn * hx2 * hy2 * lam[dir_of(i, j, 1)];
        bDxz += sgn * hx2 * hz2 * lam[dir_of(i, 1, j)];
        bDyz += sgn * hy2 * hz2 * lam[dir_of(1, i, j)];
      }
    }
  }
  float bfx = hF * bDx, bfy = hF * bDy, bfz = hF * bDz;
  const float bkxy = (wh - wn) * bDxy, bkxz = (wh - wn) * bDxz, bkyz = (wh - wn) * bDyz;
  const float bD2s = (bDxx + bDyy + bDzz) * third;
  const float bD2d1 = (bDxx - 2.0f * bDyy + bDzz) * third;
  const float bD2d2 = (bDxx + bDyy - 2.0f * bDzz) * third;
  float bRb = (wh - wx) * bD2s, bRs1 = (wh - wn) * bD2d1, bRs2 = (wh - wn) * bD2d2;
  float buxx = 0.0f, buyy = 0.0f, buzz = 0.0f;
  if constexpr (CORR != 0) {
    // corrections c = theta . g and the strain-rate solve (eq. 49)
    const float bc2s = wx * bD2s, bc2d1 = wn * bD2d1, bc2d2 = wn * bD2d2;
    const float sx = hn * (bc2d1 + bc2d2) + hx * bc2s;
    const float sy = -hn * bc2d1 + hx * bc2s;
    const float sz = -hn * bc2d2 + hx * bc2s;
    buxx -= g3 * sx * gx;
    buyy -= g3 * sy * gy;
    buzz -= g3 * sz * gz;
    float bgx = tx * sx;
    const float bgy = ty * sy, bgz = tz * sz;
    const float icsy = __builtin_amdgcn_rcpf(csy), icsz = __builtin_amdgcn_rcpf(csz);
    float bcsx = -(bgy * icsy + bgz * icsz) * gx;
    bgx -= (bgy * icsy + bgz * icsz) * csx;
    float bcsy = -bgy * gy * icsy;
    float bcsz = -bgz * gz * icsz;
    const float idet = __builtin_amdgcn_rcpf(det);
    const float bN = bgx * idet, bdet = -bgx * gx * idet;
    // cotangents of the solve's right-hand sides (they reach Rs1, Rs2, Rb, and the e terms)
    const float sRs1 = bgy * icsy - csz * cby * bN;
    const float sRs2 = bgz * icsz - csy * cbz * bN;
    const float sRb = csy * csz * bN;
    bRs1 += sRs1;
    bRs2 += sRs2;
    bRb += sRb;
    bcsz += (-cby * Rs1e + csy * Rbe) * bN + (-csx * cby + csy * cbx) * bdet;
    const float bcby = -csz * Rs1e * bN - csx * csz * bdet;
    bcsy += (-cbz * Rs2e + csz * Rbe) * bN + (-csx * cbz + csz * cbx) * bdet;
    const float bcbz = -csy * Rs2e * bN - csy * csx * bdet;
    bcsx += (-csz * cby - csy * cbz) * bdet;
    const float bcbx = csy * csz * bdet;
    buxx += g * (bcsx + bcbx);
    buyy += g * (bcby - bcsy);
    buzz += g * (bcbz - bcsz);
    if constexpr (CORR == 3) {
      // e_sr1 = tB - tA, e_sr2 = tC - tA, e_br = -(tA + tB + tC), tA = a_x u_x d_x rho, ...
      const float bes1 = 2.0f * hn * bc2d1 + sRs1, bes2 = 2.0f * hn * bc2d2 + sRs2, beb = 2.0f * hx * bc2s + sRb;
      const float btA = -(bes1 + bes2 + beb), btB = bes1 - beb, btC = bes2 - beb;
      bux += btA * ax * grx;
      buy += btB * ay * gry;
      buz += btC * az * grz;
      bgrad[0] = btA * ax * ux;
      bgrad[1] = btB * ay * uy;
      bgrad[2] = btC * az * uz;
    }
  }
  // non-equilibrium second moments
  const float sR = bRb + bRs1 + bRs2, tRy = bRb - bRs1, tRz = bRb - bRs2;
  bdrho -= 3.0f * cs2 * bRb;
  float brho = -(uxx + uyy + uzz) * bRb - (uxx - uyy) * bRs1 - (uxx - uzz) * bRs2 - ux * uy * bkxy - ux * uz * bkxz -
               uy * uz * bkyz;
  buxx -= rho * sR;
  buyy -= rho * tRy;
  buzz -= rho * tRz;
  bux += fx * sR + (0.5f * fy - rho * uy) * bkxy + (0.5f * fz - rho * uz) * bkxz;
  buy += fy * tRy + (0.5f * fx - rho * ux) * bkxy + (0.5f * fz - rho * uz) * bkyz;
  buz += fz * tRz + (0.5f * fx - rho * ux) * bkxz + (0.5f * fy - rho * uy) * bkyz;
  bfx += ux * sR + 0.5f * (uy * bkxy + uz * bkxz);
  bfy += uy * tRy + 0.5f * (ux * bkxy + uz * bkyz);
  bfz += uz * tRz + 0.5f * (ux * bkxz + uy * bkyz);
  bux += 2.0f * ux * buxx;
  buy += 2.0f * uy * buyy;
  buz += 2.0f * uz * buzz;
  // u = (j + F/2) / rho
  const float bjx = bux * irho, bjy = buy * irho, bjz = buz * irho;
  bfx += 0.5f * bjx;
  bfy += 0.5f * bjy;
  bfz += 0.5f * bjz;
  brho -= (bux * ux + buy * uy + buz * uz) * irho;
  bdrho += brho;
  // low moments are linear in df
  const float bj[3] = {bjx, r * bjy, s * bjz};
  const float bP[3] = {sR, k.c2[1] * tRy, k.c2[2] * tRz};
  const float bPxy = r * bkxy, bPxz = s * bkxz, bPyz = (r * s) * bkyz;
#pragma unroll
  for (int a = 0; a < 27; ++a) {
    const int ex = kEx[a], ey = kEy[a], ez = kEz[a];
    float v = bdrho;
    if (ex != 0) v += ex * bj[0] + bP[0];
    if (ey != 0) v += ey * bj[1] + bP[1];
    if (ez != 0) v += ez * bj[2] + bP[2];
    if (ex != 0 && ey != 0) v += (float)(ex * ey) * bPxy;
    if (ex != 0 && ez != 0) v += (float)(ex * ez) * bPxz;
    if (ey != 0 && ez != 0) v += (float)(ey * ez) * bPyz;
    if constexpr (HI) v += (1.0f - wh) * lam[a];  // the (1 - w) f term of the collision
    mu[a] = v;
  }
  gfx = bfx;
  gfy = bfy;
  gfz = bfz;
}

// ------------------------------------------------------------------ adjoint step
// The adjoint arrays are in gathered-population order: the element of slot
// (a, x) holds the cotangent of the value that node x gathers as f_a (the slot
// the forward read it from).  The node's collision-input cotangents mu are then
// stored at its own slots (aligned, as the forward stores), and the cotangents
// of its collision outputs, lambda(t+1) at its own slots (b, x), are read from
// the slots that gather them next: (b, x + ebar_b), or (opp(b), x) where that
// neighbour lies beyond a wall.  That read has the forward gather's shape
// (x-shifted loads are free there), where storing mu at the gather sources
// would need x-shifted stores (measured 12% slower on the FP16 adjoint).
__device__ __forceinline__ double wave_sum_d(double v) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
  return v;
}

// lambda(t+1) of the node's own slots, periodic: direction A's group base in
// aa_odd_groups points at the row x + ebar_opp(A) lies in, at the chunk of opp(A).
template <int I = 0>
__device__ __forceinline__ void load_next_periodic(const GroupBases<const float>& b, const Upstream& u,
                                                   float (&lam)[27]) {
  constexpr int A = issue_dir(I);
  lam[opposite_of(A)] = ld_pop<kEx[A] == 0>(b.g[group_of(A)] + (1 - kEx[A]) * kB, u.xo[kEx[A] + 1]);
  if constexpr (I + 1 < 27) load_next_periodic<I + 1>(b, u, lam);
}

template <int B = 0>
__device__ __forceinline__ void load_next_walls32(const float* __restrict__ base, const Upstream& u,
                                                  const WallFlags& w, float (&lam)[27]) {
  lam[B] = ld_pop<kEx[B] == 0>(base, downstream_slot32<B>(u, w));
  if constexpr (B + 1 < 27) load_next_walls32<B + 1>(base, u, w, lam);
}

template <int B = 0>
__device__ __forceinline__ void load_next_all(const float* __restrict__ base, const NodeCoord& c, const Consts& k,
                                              float (&lam)[27]) {
  lam[B] = base[downstream_slot<B>(c, k)];
  if constexpr (B + 1 < 27) load_next_all<B + 1>(base, c, k, lam);
}

// mu at the node's own slots: whole aligned lines, non-temporal stores.
template <int I = 0>
__device__ __forceinline__ void store_own_adj(const GroupBases<float>& d, uint32_t so, const float (&mu)[27]) {
  constexpr int A = issue_dir(I);
  st_off_nt(chunk_ptr<A>(d), so, mu[A]);
  if constexpr (I + 1 < 27) store_own_adj<I + 1>(d, so, mu);
}

// WALLS: 0 periodic (row addresses, any size), 1 walls with 32-bit offsets
// across the whole state and adjoint (both below 4 GiB), 2 general (64-bit slots).
template <int ST, int CORR, int WALLS, bool RAW, bool HI>
__global__ __launch_bounds__(256, HI ? 1 : (ST == 0 ? LBM_ADJ_WAVES_32 : LBM_ADJ_WAVES_16)) void k_step_adjoint(
    const typename Store<ST>::T* __restrict__ state, const float* __restrict__ lin, float* __restrict__ lout,
    const float* __restrict__ force, float* __restrict__ grad_force, double* __restrict__ grad_uniform,
    const float* __restrict__ drho_src, float* __restrict__ grad_rho_out, int pend, Consts k, uint32_t bpr) {
  const uint32_t lb = xcd_block(blockIdx.x, gridDim.x);
  const uint32_t bxi = lb % bpr, rowid = lb / bpr;
  // with the full corrections the rows run in y-tiles like the forward step's, so that the density
  // rows of z - 1 and z + 1 that the gradient reads are still in L2
  int y, z;
  tiled_row(rowid, (uint32_t)(CORR == 3 ? k.ytile : 1), k, y, z);
  const int x = (int)(bxi * blockDim.x + threadIdx.x);
  float gfx = 0.0f, gfy = 0.0f, gfz = 0.0f;
  // full corrections: the node's density gradient from the density field of h(t), as the step
  // computed it (block-wide, with a barrier)
  float grx = 0.0f, gry = 0.0f, grz = 0.0f;
  if constexpr (CORR == 3) {
    __shared__ float lds[3][258];
    density_gradient_block(drho_src, x, y, z, x < k.nx, k, lds, grx, gry, grz);
  }
  if (x < k.nx) {
    Upstream u;
    upstream(x, y, z, k, u);
    float df[27], lam[27], mu[27];
    WallFlags w;
    if constexpr (WALLS == 2) {
      gather_all<ST>(state, make_coord(x, y, z, k), k, df);
    } else if constexpr (WALLS == 1) {
      w = wall_flags(x, y, z, k);
      gather_walls32<ST>(state, u, w, k, df);
    } else {
      gather_periodic<ST>(pull_groups(state, u), u, k, df);
    }
    if constexpr (WALLS == 2) {
      load_next_all(lin, make_coord(x, y, z, k), k, lam);
    } else if constexpr (WALLS == 1) {
      load_next_walls32(lin, u, w, lam);
    } else {
      load_next_periodic(aa_odd_groups(lin, u), u, lam);
    }
    const int64_t nrow = ((int64_t)z * k.ny + y) * k.nx;
    float fx = k.fx, fy = k.fy, fz = k.fz;
    if (force != nullptr) {
      const float* f = force + nrow;
      fx = ld_off(f, (uint32_t)x);
      fy = ld_off(f + k.n, (uint32_t)x);
      fz = ld_off(f + 2 * k.n, (uint32_t)x);
    }
    // pend (full corrections, lagged time level): the first component of grad_rho_out holds on entry
    // the node's share of the previous call's gradient cotangent, sent back through the stencil; it
    // belongs to every population the node gathered, so it joins the node's own outputs here (read
    // before the same element is overwritten below)
    float sp = 0.0f;
    if constexpr (CORR == 3) {
      if (pend) sp = ld_off(grad_rho_out + nrow, (uint32_t)x);
    }
    float bgrad[3];
    collide_vjp<CORR, RAW, HI>(df, fx, fy, fz, k, lam, mu, gfx, gfy, gfz, grx, gry, grz, bgrad);
    if constexpr (CORR == 3) {
      if (pend) {
#pragma unroll
        for (int a = 0; a < 27; ++a) mu[a] += sp;
      }
    }
    store_own_adj(own_groups(lout, u), store_offset(u.xo[1]), mu);
    if constexpr (CORR == 3) {  // the cotangent of the node's density gradient, for k_density_vjp
      float* go = grad_rho_out + nrow;
      st_off(go, (uint32_t)x, bgrad[0]);
      st_off(go + k.n, (uint32_t)x, bgrad[1]);
      st_off(go + 2 * k.n, (uint32_t)x, bgrad[2]);
    }
    if (grad_force != nullptr) {
      float* g = grad_force + nrow;
      g[x] += gfx;
      g[k.n + x] += gfy;
      g[2 * k.n + x] += gfz;
    }
  }
  if (grad_uniform != nullptr) {
    __shared__ double part[3][4];
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const double v0 = wave_sum_d((double)gfx), v1 = wave_sum_d((double)gfy), v2 = wave_sum_d((double)gfz);
    if (lane == 0) { part[0][wave] = v0; part[1][wave] = v1; part[2][wave] = v2; }
    __syncthreads();
    if (threadIdx.x < 3) {
      double v = 0.0;
      for (int w = 0; w < (int)(blockDim.x + 63) / 64; ++w) v += part[threadIdx.x][w];
      atomicAdd(&grad_uniform[threadIdx.x], v);
    }
  }
}

// ------------------------------------------------------------------ streaming only
// The data movement of k_step_adjoint with its arithmetic left out, a measured ceiling: gather the
// state, load lambda(t+1) where the adjoint step reads it, read the force and update its gradient,
// and store mu = df + lambda at the node's own slots (same addressing, row order and block shape).
template <int ST, int WALLS>
__global__ __launch_bounds__(256) void k_adjoint_stream(const typename Store<ST>::T* __restrict__ state,
                                                        const float* __restrict__ lin, float* __restrict__ lout,
                                                        const float* __restrict__ force,
                                                        float* __restrict__ grad_force, Consts k, uint32_t bpr) {
  const uint32_t lb = xcd_block(blockIdx.x, gridDim.x);
  const uint32_t bxi = lb % bpr, rowid = lb / bpr;
  int y, z;
  tiled_row(rowid, 1u, k, y, z);
  const int x = (int)(bxi * blockDim.x + threadIdx.x);
  if (x >= k.nx) return;
  Upstream u;
  upstream(x, y, z, k, u);
  float df[27], lam[27], mu[27];
  WallFlags w;
  if constexpr (WALLS == 2) {
    gather_all<ST>(state, make_coord(x, y, z, k), k, df);
    load_next_all(lin, make_coord(x, y, z, k), k, lam);
  } else if constexpr (WALLS == 1) {
    w = wall_flags(x, y, z, k);
    gather_walls32<ST>(state, u, w, k, df);
    load_next_walls32(lin, u, w, lam);
  } else {
    gather_periodic<ST>(pull_groups(state, u), u, k, df);
    load_next_periodic(aa_odd_groups(lin, u), u, lam);
  }
#pragma unroll
  for (int a = 0; a < 27; ++a) mu[a] = df[a] + lam[a];
  store_own_adj(own_groups(lout, u), store_offset(u.xo[1]), mu);
  if (force != nullptr && grad_force != nullptr) {
    const int64_t nrow = ((int64_t)z * k.ny + y) * k.nx;
    const float* f = force + nrow;
    float* g = grad_force + nrow;
    g[x] += ld_off(f, (uint32_t)x);
    g[k.n + x] += ld_off(f + k.n, (uint32_t)x);
    g[2 * k.n + x] += ld_off(f + 2 * k.n, (uint32_t)x);
  }
}

template <int ST>
hipError_t AdjointKernels<ST>::stream(const lbm_handle& h, const void* state, const float* adj_in, float* adj_out,
                                      const float* force, float* grad_force, hipStream_t st) {
  using T = typename Store<ST>::T;
  const int block = h.block;
  const uint32_t bpr = (uint32_t)((h.p.nx + block - 1) / block);
  const int64_t nb = (int64_t)bpr * h.p.ny * h.p.nz;
  if (nb > 0x7fffffffLL) return hipErrorInvalidConfiguration;
  const bool any_wall = h.k.bb_x || h.k.bb_y || h.k.bb_z;
  const bool fits32 = 27ull * (uint64_t)h.stride * 4u < (1ull << 32);
  int kind = !any_wall ? 0 : (fits32 ? 1 : 2);
  if (h.force_kind > kind && (h.force_kind == 2 || fits32)) kind = h.force_kind;
  // the adjoint step's occupancy, 3 waves per SIMD (its registers there, reserved LDS here)
  const int blocks_per_cu = 4 * 3 / (block / 64);
  const unsigned lds = blocks_per_cu < 1 ? 0u : (unsigned)((163840 / blocks_per_cu) & ~511);
  const dim3 grid((unsigned)nb), blk(block);
  const T* s = (const T*)state;
  switch (kind) {
    case 0: hipLaunchKernelGGL((k_adjoint_stream<ST, 0>), grid, blk, lds, st, s, adj_in, adj_out, force, grad_force,
                               h.k, bpr); break;
    case 1: hipLaunchKernelGGL((k_adjoint_stream<ST, 1>), grid, blk, lds, st, s, adj_in, adj_out, force, grad_force,
                               h.k, bpr); break;
    default: hipLaunchKernelGGL((k_adjoint_stream<ST, 2>), grid, blk, lds, st, s, adj_in, adj_out, force, grad_force,
                                h.k, bpr); break;
  }
  return hipGetLastError();
}

// ------------------------------------------------------------------ launcher
template <int ST, bool HI>
static hipError_t launch_step_adjoint_t(const lbm_handle& h, const void* state, const float* adj_in, float* adj_out,
                                        const float* force, float* grad_force, double* grad_uniform,
                                        const float* drho, float* grad_rho, bool pend, hipStream_t st) {
  using T = typename Store<ST>::T;
  const int block = h.block;
  const uint32_t bpr = (uint32_t)((h.p.nx + block - 1) / block);
  const int64_t nb = (int64_t)bpr * h.p.ny * h.p.nz;
  if (nb > 0x7fffffffLL) return hipErrorInvalidConfiguration;
  const T* s = (const T*)state;
  // 32-bit offsets across all 27 chunks (walls): the float adjoint arrays below 4 GiB
  const bool any_wall = h.k.bb_x || h.k.bb_y || h.k.bb_z;
  const bool fits32 = 27ull * (uint64_t)h.stride * 4u < (1ull << 32);
  int kind = !any_wall ? 0 : (fits32 ? 1 : 2);
  if (h.force_kind > kind && (h.force_kind == 2 || fits32)) kind = h.force_kind;
  const dim3 grid((unsigned)nb), blk(block);
#define CLBM_ADJ(C, W, R)                                                                              \
  hipLaunchKernelGGL((k_step_adjoint<ST, C, W, R, HI>), grid, blk, 0, st, s, adj_in, adj_out, force, grad_force, \
                     grad_uniform, drho, grad_rho, pend ? 1 : 0, h.k, bpr)
#define CLBM_ADJ_CORR(W, R)                  \
  switch (h.p.corr) {                        \
    case 0: CLBM_ADJ(0, W, R); break;        \
    case 1: CLBM_ADJ(1, W, R); break;        \
    case 2: CLBM_ADJ(2, W, R); break;        \
    default: CLBM_ADJ(3, W, R); break;       \
  }
  const bool raw = h.p.moments == LBM_RAW;
  if (kind == 2) {
    if (raw) { CLBM_ADJ_CORR(2, true) } else { CLBM_ADJ_CORR(2, false) }
  } else if (kind == 1) {
    if (raw) { CLBM_ADJ_CORR(1, true) } else { CLBM_ADJ_CORR(1, false) }
  } else {
    if (raw) { CLBM_ADJ_CORR(0, true) } else { CLBM_ADJ_CORR(0, false) }
  }
#undef CLBM_ADJ_CORR
#undef CLBM_ADJ
  return hipGetLastError();
}

template <int ST>
hipError_t AdjointKernels<ST>::step(const lbm_handle& h, const void* state, const float* adj_in, float* adj_out,
                                    const float* force, float* grad_force, double* grad_uniform, const float* drho,
                                    float* grad_rho, bool pend, hipStream_t st) {
  return h.k.hi ? launch_step_adjoint_t<ST, true>(h, state, adj_in, adj_out, force, grad_force, grad_uniform, drho,
                                                  grad_rho, pend, st)
                : launch_step_adjoint_t<ST, false>(h, state, adj_in, adj_out, force, grad_force, grad_uniform, drho,
                                                   grad_rho, pend, st);
}

}  // namespace clbm
