"""Streaming with periodic and halfway bounce-back boundaries (oracle; test infrastructure only).

Streaming (Sec. 3.2): f_a(x, t+1) = f~_a(x - e_a, t), written in index space
(x - ebar_a), since the cuboid geometry enters only through the moments.
x is always periodic.  Along y and z the boundary is either periodic or a
stationary halfway bounce-back wall (Sec. 4 with wall velocity U = 0): when the
upstream node x - ebar_a lies outside the fluid, f_a(x, t+1) = f~_abar(x, t).
The wall then sits half a cell outside the first and last fluid node.
"""

import functools

import torch

from . import lattice as L
from .params import Params

_OPP = None


def _opp():
    global _OPP
    if _OPP is None:
        _OPP = L.opposite()
    return _OPP


@functools.lru_cache(maxsize=4096)
def outside_mask(p: Params, a):
    """Boolean (nz, ny, nx) mask of the nodes whose upstream node along a is a wall."""
    ex, ey, ez = L.EX[a], L.EY[a], L.EZ[a]
    mask = torch.zeros(p.nz, p.ny, p.nx, dtype=torch.bool)
    if p.bc_y == "bounceback" and ey != 0:
        y = torch.arange(p.ny)
        out_y = (y - ey < 0) | (y - ey >= p.ny)
        mask |= out_y[None, :, None].expand(p.nz, p.ny, p.nx)
    if p.bc_z == "bounceback" and ez != 0:
        z = torch.arange(p.nz)
        out_z = (z - ez < 0) | (z - ez >= p.nz)
        mask |= out_z[:, None, None].expand(p.nz, p.ny, p.nx)
    del ex
    return mask


def stream(ft, p: Params):
    """Pull-stream post-collision populations ``ft`` of shape (27, nz, ny, nx)."""
    opp = _opp()
    out = torch.empty_like(ft)
    for a in range(L.Q27):
        shifted = torch.roll(ft[a], shifts=(L.EZ[a], L.EY[a], L.EX[a]), dims=(0, 1, 2))
        mask = outside_mask(p, a)
        out[a] = torch.where(mask, ft[opp[a]], shifted)
    return out
