"""Equilibria and source moments (oracle; test infrastructure only).

* central-moment equilibria matched to the Maxwellian, eq. 9
* raw-moment equilibria, eq. 10, obtained here as F(-u) applied to eq. 9
  (the binomial transform the paper names); a test checks them against eq. 10
* equilibrium populations f_eq = Q^-1 m_eq (Sec. 4 uses the same map for the
  wall equilibria)
* central source moments, eq. 11c
"""

import torch

from . import lattice as L

DT = L.DT


def central_equilibrium(rho, cs2):
    """m^{c,eq} of eq. 9 in the MOMENTS ordering; ``rho`` shape (N,), result (N, 27).

    k_000 = rho; k_200 = k_020 = k_002 = cs2 rho; k_220 = k_202 = k_022 = cs2^2 rho;
    k_222 = cs2^3 rho; every other central moment is zero.
    """
    out = torch.zeros(rho.shape[0], L.Q27, dtype=rho.dtype)
    out[:, L.MIDX[(0, 0, 0)]] = rho
    for mnp in ((2, 0, 0), (0, 2, 0), (0, 0, 2)):
        out[:, L.MIDX[mnp]] = cs2 * rho
    for mnp in ((2, 2, 0), (2, 0, 2), (0, 2, 2)):
        out[:, L.MIDX[mnp]] = cs2 ** 2 * rho
    out[:, L.MIDX[(2, 2, 2)]] = cs2 ** 3 * rho
    return out


def raw_equilibrium(rho, u, cs2):
    """m^{eq} (cuboid raw moments): F(-u) m^{c,eq}; equals eq. 10 (checked by a test)."""
    return torch.einsum("nab,nb->na", L.frame_matrix_inverse(u), central_equilibrium(rho, cs2))


def feq(rho, u, r, s, cs2):
    """Equilibrium populations f_eq = Q^-1 m_eq = P^-1 S^-1 m_eq, shape (N, 27)."""
    m = raw_equilibrium(rho, u, cs2)
    m = m / L.S_diag(r, s)
    return m @ L.P_inverse().T


def central_source(force):
    """Phi^c of eq. 11c: sigma_100, sigma_010, sigma_001 = F; all others 0. (N, 27)."""
    out = torch.zeros(force.shape[0], L.Q27, dtype=force.dtype)
    out[:, L.MIDX[(1, 0, 0)]] = force[:, 0]
    out[:, L.MIDX[(0, 1, 0)]] = force[:, 1]
    out[:, L.MIDX[(0, 0, 1)]] = force[:, 2]
    return out


def rest_weights(r, s, cs2):
    """w_alpha = f_eq(rho = 1, u = 0): the rest-state weights (shape (27,))."""
    one = torch.ones(1, dtype=DT)
    zero = torch.zeros(1, 3, dtype=DT)
    return feq(one, zero, r, s, cs2)[0]
