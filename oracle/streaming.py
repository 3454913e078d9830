"""Streaming with periodic and halfway bounce-back boundaries (oracle; test infrastructure only).

Streaming (Sec. 3.2): f_a(x, t+1) = f~_a(x - e_a, t), written in index space
(x - ebar_a), since the cuboid geometry enters only through the moments.
Each axis is periodic or bounded by halfway bounce-back walls, which sit half a
cell outside the first and last fluid node.  When the upstream node x - ebar_a
lies outside the fluid, the momentum-augmented bounce-back of Sec. 4 applies:
    f_a(x, t+1) = f~_abar(x, t) - [f_eq_abar(x_w) - f_eq_a(x_w)],
with the wall equilibrium f_eq = Q^-1 m_eq (eq. 10) at the wall velocity and
the density of the fluid node, rho_w = rho(x, t) = sum_b f~_b(x, t).  For a wall
moving along x this is eq. 69; for a stationary wall the bracket vanishes.  A
link that leaves through two or three faces at once (an edge or corner of the
box) takes the mean velocity of the moving faces among them (zero if none
moves): a lid then meets the side walls without a mass source, since the wall
terms of each node cancel in pairs.
"""

import functools

import torch

from . import equilibrium as EQ
from . import lattice as L
from .params import Params

_OPP = None


def _opp():
    global _OPP
    if _OPP is None:
        _OPP = L.opposite()
    return _OPP


@functools.lru_cache(maxsize=4096)
def wall_link(p: Params, a):
    """(mask, velocity) of the wall links of direction a: mask (nz, ny, nx) marks the
    nodes whose upstream node x - ebar_a is outside the fluid; velocity (3, nz, ny, nx)
    is the mean velocity of the moving faces that link crosses (zero elsewhere)."""
    e = (L.EX[a], L.EY[a], L.EZ[a])
    bcs = (p.bc_x, p.bc_y, p.bc_z)
    sizes = (p.nx, p.ny, p.nz)
    dims = (2, 1, 0)                       # tensor dimension of axis x, y, z
    crossed = torch.zeros(p.nz, p.ny, p.nx, dtype=torch.bool)
    count = torch.zeros(p.nz, p.ny, p.nx, dtype=L.DT)        # moving faces crossed
    vel = torch.zeros(3, p.nz, p.ny, p.nx, dtype=L.DT)
    for d in range(3):
        if bcs[d] != "bounceback" or e[d] == 0:
            continue
        idx = torch.arange(sizes[d])
        for side, hit in ((0, idx - e[d] < 0), (1, idx - e[d] >= sizes[d])):
            shape = [1, 1, 1]
            shape[dims[d]] = sizes[d]
            h = hit.reshape(shape).expand(p.nz, p.ny, p.nx).to(L.DT)
            crossed |= h > 0
            u = p.wall_velocity[2 * d + side]
            if any(c != 0.0 for c in u):
                count += h
                for c in range(3):
                    vel[c] += h * u[c]
    vel = vel / count.clamp(min=1.0)[None]
    return crossed, vel


def outside_mask(p: Params, a):
    """Boolean (nz, ny, nx) mask of the nodes whose upstream node along a is a wall."""
    return wall_link(p, a)[0]


def stream(ft, p: Params):
    """Pull-stream post-collision populations ``ft`` of shape (27, nz, ny, nx)."""
    opp = _opp()
    out = torch.empty_like(ft)
    moving = any(any(c != 0.0 for c in v) for v in p.wall_velocity)
    rho_w = ft.sum(0) if moving else None
    for a in range(L.Q27):
        shifted = torch.roll(ft[a], shifts=(L.EZ[a], L.EY[a], L.EX[a]), dims=(0, 1, 2))
        mask, vel = wall_link(p, a)
        out[a] = torch.where(mask, ft[opp[a]], shifted)
        if moving and bool(mask.any()):
            u = vel[:, mask].T                                     # (M, 3) wall velocities of the links
            feq = EQ.feq(rho_w[mask], u, p.r, p.s, p.cs2)          # wall equilibria, rho_w = rho of the fluid node
            out[a][mask] = out[a][mask] - (feq[:, opp[a]] - feq[:, a])
    return out
