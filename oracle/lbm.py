"""Initialisation, time step and observables of the oracle (test infrastructure only).

One step is collide (Sec. 3.2, App. A-G) followed by streaming with the
boundary conditions of Sec. 4 (stationary walls).  The state between steps is
the post-stream population field f(x, t), laid out (27, nz, ny, nx); node
index = (z * ny + y) * nx + x.  Observables follow eq. 12 (also the last
bullet of Sec. 3.2).
"""

import torch

from . import collision as C
from . import equilibrium as EQ
from . import lattice as L
from . import streaming as ST
from .params import Params  # noqa: F401  (re-exported)

DT = L.DT
CHUNK = 32768


def to_nodes(f):
    """(27, nz, ny, nx) -> (N, 27)."""
    return f.reshape(L.Q27, -1).T


def from_nodes(fn, p: Params):
    """(N, 27) -> (27, nz, ny, nx)."""
    return fn.T.reshape(L.Q27, p.nz, p.ny, p.nx)


def force_nodes(force, p: Params):
    """Force as (N, 3): None -> 0, a 3-sequence -> uniform, a (3, nz, ny, nx) field."""
    if force is None:
        return torch.zeros(p.n, 3, dtype=DT)
    force = torch.as_tensor(force, dtype=DT)
    if force.dim() == 1:
        return force[None, :].expand(p.n, 3)
    return force.reshape(3, -1).T


def init_equilibrium(rho, u, p: Params):
    """f(x, 0) = f_eq(rho, u) (eq. 9 mapped to populations); rho (nz,ny,nx), u (3,nz,ny,nx)."""
    rho_n = torch.as_tensor(rho, dtype=DT).reshape(-1)
    u_n = torch.as_tensor(u, dtype=DT).reshape(3, -1).T
    out = []
    for i in range(0, p.n, CHUNK):
        out.append(EQ.feq(rho_n[i:i + CHUNK], u_n[i:i + CHUNK], p.r, p.s, p.cs2))
    return from_nodes(torch.cat(out), p)


def density_gradient(rho, p: Params):
    """Second-order central differences of rho with spacings (1, r, s).

    Only the "full" correction variant uses it.  Periodic axes wrap; at a
    bounce-back wall the first/last node uses the one-sided second-order
    difference.  The paper names an isotropic second-order stencil without
    fixing it: parity unpinned.
    """
    out = []
    for axis, h, bc in ((2, 1.0, "periodic"), (1, p.r, p.bc_y), (0, p.s, p.bc_z)):
        n = rho.shape[axis]
        g = (torch.roll(rho, -1, axis) - torch.roll(rho, 1, axis)) / (2 * h)
        if bc == "bounceback" and n >= 3:
            idx = torch.arange(n)
            first = (-3 * rho.index_select(axis, idx[0:1]) + 4 * rho.index_select(axis, idx[1:2])
                     - rho.index_select(axis, idx[2:3])) / (2 * h)
            last = (3 * rho.index_select(axis, idx[-1:]) - 4 * rho.index_select(axis, idx[-2:-1])
                    + rho.index_select(axis, idx[-3:-2])) / (2 * h)
            g = g.clone()
            g.index_copy_(axis, idx[0:1], first)
            g.index_copy_(axis, idx[-1:], last)
        out.append(g)
    return torch.stack(out)  # (3, nz, ny, nx): d/dx, d/dy, d/dz


def collide_field(f, p: Params, force=None):
    """Collision on every node of a (27, nz, ny, nx) field."""
    fn = to_nodes(f)
    Fn = force_nodes(force, p)
    grad = None
    if p.corr == "full":
        rho = f.sum(0)
        grad = density_gradient(rho, p).reshape(3, -1).T
    out = []
    for i in range(0, p.n, CHUNK):
        g = None if grad is None else grad[i:i + CHUNK]
        out.append(C.collide(fn[i:i + CHUNK], Fn[i:i + CHUNK], p, grad_rho=g))
    return from_nodes(torch.cat(out), p)


def step(f, p: Params, force=None):
    """One collide-and-stream step: f(t) -> f(t + 1)."""
    return ST.stream(collide_field(f, p, force), p)


def run(f, p: Params, nsteps, force=None):
    for _ in range(nsteps):
        f = step(f, p, force)
    return f


def observables(f, p: Params, force=None):
    """rho (nz, ny, nx) and u (3, nz, ny, nx) of eq. 12 for a post-stream field."""
    rho, u = C.macroscopic(to_nodes(f), force_nodes(force, p), p)
    return rho.reshape(p.shape), u.T.reshape(3, *p.shape)


def sums(f, p: Params, force=None):
    """FP64 totals: mass, momentum x/y/z, kinetic energy sum 0.5 rho |u|^2 (per node)."""
    rho, u = observables(f, p, force)
    mom = (rho[None] * u).reshape(3, -1).sum(-1)
    energy = 0.5 * (rho[None] * u * u).sum()
    return torch.stack([rho.sum(), mom[0], mom[1], mom[2], energy])
