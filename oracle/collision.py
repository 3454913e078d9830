"""Collision step of the 3DCCM-LBM (oracle; test infrastructure only).

Follows the bullet list of Sec. 3.2 in order, with explicit 27x27 matrices:

  m = P f                         (App. A)
  m <- S m                        (App. B)
  m^c = F(u) m                    (App. C)
  n = B m^c; strain rates; effective equilibria; relaxation with sources (App. D)
  m~^c = B^-1 n~                  (segregation at the end of App. D)
  m~ = F(-u) m~^c                 (App. E)
  m~ <- S^-1 m~                   (App. F)
  f~ = P^-1 m~                    (App. G)

The velocity is the force-shifted one of eq. 12: rho u = sum f e + F/2.
With ``moments="raw"`` the relaxation acts on the raw moments instead (the
raw-moment scheme of Sec. 7; ``relax_raw``).
Readings where the paper is silent or garbled (see the design notes):
* the non-equilibrium moments of the strain-rate solve are the pre-collision
  central moments minus the *uncorrected* equilibria (eq. 45-46);
* "lowmach" drops the 3u^2 terms both in theta and in the strain-rate
  coefficients C (the non-Galilean-invariant terms neglected together);
* "full" takes the density gradient as an input; "local"/"lowmach" set it to 0.
"""

import torch

from . import lattice as L
from . import equilibrium as EQ
from .params import Params

DT = L.DT


def relaxation_diag(p: Params):
    """Diagonal of Lambda in the n ordering (App. D, rates other than nu/xi = omega_hi)."""
    lam = torch.full((L.Q27,), float(p.omega_hi), dtype=DT)
    lam[0] = 1.0                                  # k_000: conserved, rate irrelevant
    lam[1:4] = p.omega_1
    lam[4:7] = p.omega_nu                         # k_110, k_101, k_011
    lam[L.N_2D1] = p.omega_nu
    lam[L.N_2D2] = p.omega_nu
    lam[L.N_2S] = p.omega_xi
    return lam


def strain_rates(n, rho, u, p: Params, grad_rho):
    """Diagonal strain rates d_x u_x, d_y u_y, d_z u_z from the local 3x3 system (App. D).

    ``n`` are the combined pre-collision central moments (n ordering).  The
    system C . du = R is built from C_sx ... C_bz and R_s1, R_s2, R_b exactly as
    App. D (eq. 44-48) defines them and solved densely (eq. 49 / eq. 65 give its
    closed-form solution).  Returns (N, 3).
    """
    cs2, r2, s2 = p.cs2, p.r ** 2, p.s ** 2
    ux, uy, uz = u[:, 0], u[:, 1], u[:, 2]
    g = 0.0 if p.corr == "lowmach" else 1.0       # weight of the 3u^2 (non-GI) terms
    # e_rho terms (zero unless the density gradient is supplied)
    A = 0.5 * (3 * cs2 - 1.0) * ux
    Bc = 0.5 * (3 * cs2 - r2) * uy
    Cc = 0.5 * (3 * cs2 - s2) * uz
    dxr, dyr, dzr = grad_rho[:, 0], grad_rho[:, 1], grad_rho[:, 2]
    e_sr1 = -A * dxr + Bc * dyr
    e_sr2 = -A * dxr + Cc * dzr
    e_br = -A * dxr - Bc * dyr - Cc * dzr
    R_b = n[:, L.N_2S] - 3 * cs2 * rho + e_br
    R_s1 = n[:, L.N_2D1] + e_sr1
    R_s2 = n[:, L.N_2D2] + e_sr2
    wn, wx = p.omega_nu, p.omega_xi
    C_sx = (-2 * cs2 / wn + 0.5 * (3 * cs2 - 1.0) + g * 1.5 * ux ** 2) * rho
    C_bx = (-2 * cs2 / wx + 0.5 * (3 * cs2 - 1.0) + g * 1.5 * ux ** 2) * rho
    C_sy = (2 * cs2 / wn - 0.5 * (3 * cs2 - r2) - g * 1.5 * uy ** 2) * rho
    C_by = (-2 * cs2 / wx + 0.5 * (3 * cs2 - r2) + g * 1.5 * uy ** 2) * rho
    C_sz = (2 * cs2 / wn - 0.5 * (3 * cs2 - s2) - g * 1.5 * uz ** 2) * rho
    C_bz = (-2 * cs2 / wx + 0.5 * (3 * cs2 - s2) + g * 1.5 * uz ** 2) * rho
    zero = torch.zeros_like(rho)
    M = torch.stack([
        torch.stack([C_sx, C_sy, zero], -1),
        torch.stack([C_sx, zero, C_sz], -1),
        torch.stack([C_bx, C_by, C_bz], -1),
    ], -2)
    det = torch.linalg.det(M)
    if bool(torch.any(det.abs() <= 1e-12 * rho.abs() ** 3)):
        raise FloatingPointError("strain-rate system singular (|det| <= 1e-12 rho^3)")
    R = torch.stack([R_s1, R_s2, R_b], -1)
    return torch.linalg.solve(M, R.unsqueeze(-1)).squeeze(-1)


def correction_terms(rho, u, du, p: Params, grad_rho):
    """Corrections added to k_2d1^eq, k_2d2^eq, k_2s^eq (App. D, eq. 38-40); (N, 3)."""
    zero = torch.zeros_like(rho)
    if p.corr == "off":
        return torch.stack([zero, zero, zero], -1)
    cs2, r2, s2 = p.cs2, p.r ** 2, p.s ** 2
    ux, uy, uz = u[:, 0], u[:, 1], u[:, 2]
    g = 0.0 if p.corr == "lowmach" else 1.0
    hn = 1.0 / p.omega_nu - 0.5
    hx = 1.0 / p.omega_xi - 0.5
    th_sx = -rho * (g * 3 * ux ** 2 + 3 * cs2 - 1.0) * hn
    th_bx = -rho * (g * 3 * ux ** 2 + 3 * cs2 - 1.0) * hx
    th_sy = -rho * (g * 3 * uy ** 2 + 3 * cs2 - r2) * hn
    th_by = -rho * (g * 3 * uy ** 2 + 3 * cs2 - r2) * hx
    th_sz = -rho * (g * 3 * uz ** 2 + 3 * cs2 - s2) * hn
    th_bz = -rho * (g * 3 * uz ** 2 + 3 * cs2 - s2) * hx
    dxux, dyuy, dzuz = du[:, 0], du[:, 1], du[:, 2]
    c2d1 = th_sx * dxux - th_sy * dyuy
    c2d2 = th_sx * dxux - th_sz * dzuz
    c2s = th_bx * dxux + th_by * dyuy + th_bz * dzuz
    if p.corr == "full":
        la_sx = -(3 * cs2 - 1.0) * hn * ux
        la_bx = -(3 * cs2 - 1.0) * hx * ux
        la_sy = (3 * cs2 - r2) * hn * uy
        la_by = -(3 * cs2 - r2) * hx * uy
        la_sz = (3 * cs2 - s2) * hn * uz
        la_bz = -(3 * cs2 - s2) * hx * uz
        dxr, dyr, dzr = grad_rho[:, 0], grad_rho[:, 1], grad_rho[:, 2]
        c2d1 = c2d1 + la_sx * dxr + la_sy * dyr
        c2d2 = c2d2 + la_sx * dxr + la_sz * dzr
        c2s = c2s + la_bx * dxr + la_by * dyr + la_bz * dzr
    return torch.stack([c2d1, c2d2, c2s], -1)


def macroscopic(f, force, p: Params):
    """rho and u of eq. 12 (dt = 1): rho = sum f, rho u = sum f e + F/2.  f: (N, 27)."""
    e = L.velocities(p.r, p.s)
    rho = f.sum(-1)
    u = (f @ e + 0.5 * force) / rho[:, None]
    return rho, u


def relax_central(mc, rho, u, force, p: Params, grad_rho):
    """Post-collision central moments from pre-collision ones (App. D).

    B combines, the strain rates and the effective equilibria follow, every
    combined moment relaxes with its rate and the source enters as
    (I - Lambda/2) B Phi^c; B^-1 segregates.  Returns (m~^c, strain rates).
    """
    n_nodes = mc.shape[0]
    B, Binv = L.B_matrix(), L.B_inverse()
    nvec = mc @ B.T
    if p.corr == "off":
        du = torch.zeros(n_nodes, 3, dtype=mc.dtype)
    else:
        du = strain_rates(nvec, rho, u, p, grad_rho)
    n_eq = EQ.central_equilibrium(rho, p.cs2) @ B.T
    corr = correction_terms(rho, u, du, p, grad_rho)
    n_eq = n_eq.clone()
    n_eq[:, L.N_2D1] = n_eq[:, L.N_2D1] + corr[:, 0]
    n_eq[:, L.N_2D2] = n_eq[:, L.N_2D2] + corr[:, 1]
    n_eq[:, L.N_2S] = n_eq[:, L.N_2S] + corr[:, 2]
    lam = relaxation_diag(p)
    phi = EQ.central_source(force) @ B.T
    n_post = nvec + lam * (n_eq - nvec) + (1.0 - 0.5 * lam) * phi
    return n_post @ Binv.T, du


def relax_raw(m, mc, rho, u, force, p: Params, grad_rho):
    """Post-collision raw moments of the raw-moment scheme (3DCRM-LBM, Sec. 7).

    The relaxation of the combined moments (App. D) acts on raw moments: the
    raw equilibria are F(-u) applied to the central ones (eq. 10), the
    corrections enter the same combined second-order equilibria, and the
    source is the raw image F(-u) Phi^c of the central source of eq. 11c.
    The strain rates of the corrections are taken from the central moments
    ``mc`` exactly as in the central scheme.  Returns (m~, strain rates).
    """
    n_nodes = m.shape[0]
    B, Binv = L.B_matrix(), L.B_inverse()
    Finv = L.frame_matrix_inverse(u)
    if p.corr == "off":
        du = torch.zeros(n_nodes, 3, dtype=m.dtype)
    else:
        du = strain_rates(mc @ B.T, rho, u, p, grad_rho)
    m_eq = torch.einsum("nab,nb->na", Finv, EQ.central_equilibrium(rho, p.cs2))
    n_eq = (m_eq @ B.T).clone()
    corr = correction_terms(rho, u, du, p, grad_rho)
    n_eq[:, L.N_2D1] = n_eq[:, L.N_2D1] + corr[:, 0]
    n_eq[:, L.N_2D2] = n_eq[:, L.N_2D2] + corr[:, 1]
    n_eq[:, L.N_2S] = n_eq[:, L.N_2S] + corr[:, 2]
    phi = torch.einsum("nab,nb->na", Finv, EQ.central_source(force)) @ B.T
    lam = relaxation_diag(p)
    nvec = m @ B.T
    n_post = nvec + lam * (n_eq - nvec) + (1.0 - 0.5 * lam) * phi
    return n_post @ Binv.T, du


def collide(f, force, p: Params, grad_rho=None, return_info=False):
    """Post-collision populations f~ for populations ``f`` (N, 27) and force (N, 3)."""
    n_nodes = f.shape[0]
    if grad_rho is None or p.corr != "full":
        grad_rho = torch.zeros(n_nodes, 3, dtype=f.dtype)
    Pm, Pinv = L.P_matrix(), L.P_inverse()
    S = L.S_diag(p.r, p.s)

    # pre-collision raw moments on the cubic lattice, then scaled to the cuboid one
    m = f @ Pm.T
    m = m * S
    rho = m[:, L.MIDX[(0, 0, 0)]]
    j = torch.stack([m[:, L.MIDX[(1, 0, 0)]], m[:, L.MIDX[(0, 1, 0)]], m[:, L.MIDX[(0, 0, 1)]]], -1)
    u = (j + 0.5 * force) / rho[:, None]

    # pre-collision central moments
    mc = torch.einsum("nab,nb->na", L.frame_matrix(u), m)

    if p.moments == "raw":
        # relaxation of raw moments (no frame transformation around the collision)
        m_post, du = relax_raw(m, mc, rho, u, force, p, grad_rho)
        mc_post = torch.einsum("nab,nb->na", L.frame_matrix(u), m_post)
    else:
        # relaxation in central-moment space (B, strain rates, extended equilibria, B^-1)
        mc_post, du = relax_central(mc, rho, u, force, p, grad_rho)
        # back to raw moments
        m_post = torch.einsum("nab,nb->na", L.frame_matrix_inverse(u), mc_post)

    # unscale, back to populations
    m_post = m_post / S
    f_post = m_post @ Pinv.T
    if return_info:
        return f_post, {"rho": rho, "u": u, "du": du, "mc": mc, "mc_post": mc_post}
    return f_post
