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
    """Isotropic second-order density gradient on the cuboid lattice (App. D).

    App. D takes d_x rho, d_y rho, d_z rho from an isotropic second-order
    finite-difference stencil without printing it.  The stencil here is the
    lattice-weighted one,
        grad rho (x) = (1 / cs2) sum_a w_a e_a rho(x + ebar_a),
    with the rest weights w_a and the cuboid velocities e_a = (ebar_x, r ebar_y,
    s ebar_z); because sum_a w_a e_a e_a = cs2 I, it is exact for fields of
    degree <= 2 and its leading error is isotropic.  Periodic axes wrap; across
    a halfway bounce-back wall the neighbour is the mirror image of the node
    across the wall, i.e. the boundary node itself (the index is clamped).
    Returns (3, nz, ny, nx): d/dx, d/dy, d/dz.
    """
    rho = torch.as_tensor(rho, dtype=DT)
    w = EQ.rest_weights(p.r, p.s, p.cs2)
    e = L.velocities(p.r, p.s)
    ebar = L.velocities(1.0, 1.0).round().to(torch.int64)
    idx = []
    for n, bc in ((p.nz, p.bc_z), (p.ny, p.bc_y), (p.nx, p.bc_x)):
        base = torch.arange(n)
        idx.append({d: (torch.clamp(base + d, 0, n - 1) if bc == "bounceback" else (base + d) % n)
                    for d in (-1, 0, 1)})
    out = torch.zeros((3, *rho.shape), dtype=DT)
    for a in range(L.Q27):
        ex, ey, ez = (int(v) for v in ebar[a])
        nb = rho.index_select(0, idx[0][ez]).index_select(1, idx[1][ey]).index_select(2, idx[2][ex])
        for d in range(3):
            out[d] += w[a] * e[a, d] * nb
    return out / p.cs2


def collide_field(f, p: Params, force=None, grad_from=None):
    """Collision on every node of a (27, nz, ny, nx) field.

    With the "full" corrections the density gradient is taken from
    ``grad_from`` (a density field) when given, else from the density of ``f``.
    """
    fn = to_nodes(f)
    Fn = force_nodes(force, p)
    grad = None
    if p.corr == "full":
        rho = f.sum(0) if grad_from is None else torch.as_tensor(grad_from, dtype=DT)
        grad = density_gradient(rho, p).reshape(3, -1).T
    out = []
    for i in range(0, p.n, CHUNK):
        g = None if grad is None else grad[i:i + CHUNK]
        out.append(C.collide(fn[i:i + CHUNK], Fn[i:i + CHUNK], p, grad_rho=g))
    return from_nodes(torch.cat(out), p)


def step(f, p: Params, force=None, grad_from=None):
    """One collide-and-stream step: f(t) -> f(t + 1)."""
    return ST.stream(collide_field(f, p, force, grad_from), p)


def run(f, p: Params, nsteps, force=None, lagged=False):
    """nsteps steps.  ``lagged`` (full corrections only): the first step takes its
    density gradient from the density of its own input, every later step from the
    density of the previous step's input (one step behind)."""
    prev = None
    for _ in range(nsteps):
        now = f.sum(0) if (lagged and p.corr == "full") else None
        f = step(f, p, force, prev if lagged else None)
        prev = now
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
