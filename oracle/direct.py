"""Independent route to the collision through the definition of central moments.

Test infrastructure only.  The central moments of eq. 3a are formed directly
as k_mnp = sum_a f_a (e_ax - u_x)^m (e_ay - u_y)^n (e_az - u_z)^p with the
cuboid velocities, and the post-collision populations are recovered by a
dense solve of the same 27x27 system.  This shares the relaxation in
central-moment space (App. D) with ``collision`` but none of the factors
P, S, F(u), their inverses or App. A-C/E-G; comparing the two pins that
factor chain.
"""

import torch

from . import lattice as L
from . import collision as C
from .params import Params


def central_moment_matrix(u, r, s):
    """M_c(u)[k, a] = (e_a - u)^(m,n,p) for each node: shape (N, 27, 27)."""
    e = L.velocities(r, s)                       # (27, 3)
    d = e[None, :, :] - u[:, None, :]            # (N, 27, 3)
    rows = [d[:, :, 0] ** m * d[:, :, 1] ** n * d[:, :, 2] ** p for (m, n, p) in L.MOMENTS]
    return torch.stack(rows, 1)


def collide(f, force, p: Params, grad_rho=None):
    """Same collision as ``collision.collide`` computed through eq. 3a and a dense solve."""
    if grad_rho is None or p.corr != "full":
        grad_rho = torch.zeros(f.shape[0], 3, dtype=f.dtype)
    e = L.velocities(p.r, p.s)
    rho = f.sum(-1)
    u = (f @ e + 0.5 * force) / rho[:, None]
    M = central_moment_matrix(u, p.r, p.s)
    mc = torch.einsum("nka,na->nk", M, f)
    mc_post, _ = C.relax_central(mc, rho, u, force, p, grad_rho)
    return torch.linalg.solve(M, mc_post.unsqueeze(-1)).squeeze(-1)
