"""GPU parity of the wall kernels' 64-bit slot path, taken when a state (or,
for the adjoint, the FP32 adjoint arrays) with walls is 4 GiB or larger:
ducts with walls in y and z, 512x512x160 (FP32 and FP16 adjoint) and
512x512x320 (FP16 step), one forward step and one adjoint step, compared
with the FP64 oracle on sampled nodes (interior, faces, edges and corners).

The oracle side is local.  Forward: the new population f_a(y) is the collided
population a of node y - ebar_a, or, when that node lies beyond a wall, the
collided population abar of y itself (halfway bounce-back, Sec. 4).  Adjoint:
the cotangent of the state at y is the transpose of y's collision applied to
mu(y), where mu_c(y) is the output cotangent at the slot that population c of
y streams to: lambda_c(y + ebar_c), or lambda_cbar(y) across a wall."""

import sys

import numpy as np
import pytest
import torch

import oracle
from oracle import collision as C
from oracle import lattice as LT
import workloads as W
import paper_2107_14774_amd as P
from helpers import gpu_lattice

pytestmark = pytest.mark.gpu
DT = torch.float64
NX, NY = 512, 512
FORCE = (2e-6, -1e-6, 5e-7)


def _say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def _params(nz):
    return oracle.Params(NX, NY, nz, r=1.0, s=0.5, omega_nu=1.45, omega_xi=1.2, corr="local",
                         bc_y="bounceback", bc_z="bounceback")


def _samples(seed, NZ):
    """48 seeded interior nodes plus face, edge and corner nodes, as (z, y, x) arrays."""
    g = np.random.Generator(np.random.PCG64(seed))
    z = list(g.integers(1, NZ - 1, 48))
    y = list(g.integers(1, NY - 1, 48))
    x = list(g.integers(0, NX, 48))
    for zz, yy in ((0, 7), (NZ - 1, 300), (40, 0), (90, NY - 1), (0, 0), (0, NY - 1), (NZ - 1, 0),
                   (NZ - 1, NY - 1)):
        for xx in (0, 255, NX - 1):
            z.append(zz)
            y.append(yy)
            x.append(xx)
    return np.array(z), np.array(y), np.array(x)


def _smooth_velocity(p, seed):
    u = torch.from_numpy(W.random_modes(p.nx, p.ny, p.nz, p.r, p.s, 3, 0.02, seed))
    return u


def _state(lat, p, seed):
    a = lat.new_state()
    lat.init(a, u=_smooth_velocity(p, seed).cuda())
    return a


def _rest_weights(p):
    from oracle import equilibrium as EQ
    return EQ.rest_weights(p.r, p.s, p.cs2)


def _gather_nodes(full, zs, ys, xs):
    """Populations (N, 27) of the nodes (zs, ys, xs) from a (27, nz, ny, nx) GPU field."""
    idx = torch.from_numpy(np.stack([zs, ys, xs])).cuda()
    return full[:, idx[0], idx[1], idx[2]].T.cpu()


@pytest.mark.parametrize("storage,nz,field", [("f32", 160, False), ("f16", 320, False), ("f32", 160, True)])
def test_large_duct_step_matches_oracle(storage, nz, field):
    """field: a force field (N floats per component, read with 64-bit indices on this path)."""
    NZ = nz
    p = _params(nz)
    lat = gpu_lattice(p, storage=storage, force=FORCE)
    assert lat.h.state_bytes >= 1 << 32                      # the 32-bit wall path ends at 4 GiB
    a = _state(lat, p, 61)
    b = lat.new_state()
    f0 = lat.export_populations(a)
    ffield = None
    if field:
        g = np.random.Generator(np.random.PCG64(63))
        ffield = torch.from_numpy((1e-5 * g.standard_normal((3, NZ, NY, NX))).astype(np.float32)).cuda()
    cur, _ = lat.step(a, b, 1, ffield)
    f1 = lat.export_populations(cur)
    zs, ys, xs = _samples(62, NZ)
    got = _gather_nodes(f1, zs, ys, xs)                      # (S, 27)
    eb = LT.ebar().numpy()
    opp = LT.opposite()
    # source node of every (sample, direction), or the sample itself across a wall
    sz = zs[:, None] - eb[None, :, 2]
    sy = ys[:, None] - eb[None, :, 1]
    sx = (xs[:, None] - eb[None, :, 0]) % NX
    wall = (sz < 0) | (sz >= NZ) | (sy < 0) | (sy >= NY)
    sz = np.where(wall, zs[:, None], sz)
    sy = np.where(wall, ys[:, None], sy)
    sx = np.where(wall, xs[:, None], sx)
    comp = np.where(wall, np.array(opp)[None, :], np.arange(27)[None, :])
    fs = _gather_nodes(f0, sz.ravel(), sy.ravel(), sx.ravel())        # (S*27, 27)
    if field:                                                           # the force of the colliding node
        force = _gather_nodes(ffield, sz.ravel(), sy.ravel(), sx.ravel()).to(DT)
    else:
        force = torch.tensor([FORCE] * fs.shape[0], dtype=DT)
    ft = C.collide(fs, force, p)
    want = ft[torch.arange(fs.shape[0]), torch.from_numpy(comp.ravel())].reshape(got.shape)
    err = (got - want).abs().max().item()
    dev = (want - _rest_weights(p).to(want.dtype)).abs().max().item()
    nwall = int(wall.any(1).sum())
    _say(f"512x512x{NZ} duct {storage}{' + force field' if field else ''} (state {lat.h.state_bytes / 2**30:.2f} GiB), "
         f"one step, {len(zs)} sampled "
         f"nodes ({nwall} next to a wall): max |f_gpu - f_oracle| = {err:.3e} (max deviation {dev:.2e})")
    assert nwall >= 24
    if storage == "f32":
        assert err < 2e-7
    else:
        # 11 significand bits on the stored deviation; a wrong source would be off by O(dev)
        assert err < 2e-3 * dev


@pytest.mark.parametrize("storage,field", [("f32", False), ("f16", False), ("f32", True)])
def test_large_duct_adjoint_matches_oracle(storage, field):
    """field: a force field and its per-node gradient (N floats per component, 64-bit indices here)."""
    NZ = 160
    p = _params(NZ)
    lat = gpu_lattice(p, storage=storage, force=FORCE)
    assert 27 * lat.h.stride * 4 >= 1 << 32                  # FP32 adjoint arrays of 4 GiB or more
    st = _state(lat, p, 63)
    f0 = lat.export_populations(st)
    g = torch.Generator(device="cuda")
    g.manual_seed(64)
    lam = torch.randn((27, NZ, NY, NX), dtype=DT, device="cuda", generator=g)
    lam_in, lam_out = lat.new_adjoint(zero=False), lat.new_adjoint()
    P.lbm_adjoint_from_natural(lat.h, lam, lam_in)
    gFu = torch.zeros(3, dtype=torch.float64, device="cuda")
    ffield = gfield = None
    if field:
        gf = np.random.Generator(np.random.PCG64(66))
        ffield = torch.from_numpy((1e-5 * gf.standard_normal((3, NZ, NY, NX))).astype(np.float32)).cuda()
        gfield = torch.zeros((3, NZ, NY, NX), dtype=torch.float32, device="cuda")
    P.lbm_step_adjoint(lat.h, st, lam_in, lam_out, ffield, gfield, gFu)
    out = torch.empty((27, NZ, NY, NX), dtype=DT, device="cuda")
    P.lbm_adjoint_to_natural(lat.h, lam_out, out)
    lam32 = lam.to(torch.float32).to(DT)                     # the kernel reads lambda in FP32
    del lam
    zs, ys, xs = _samples(65, NZ)
    got = _gather_nodes(out, zs, ys, xs)
    eb = LT.ebar().numpy()
    opp = np.array(LT.opposite())
    # mu_c(y): lambda_c at y + ebar_c, or lambda_cbar at y when y + ebar_c lies beyond a wall
    tz = zs[:, None] + eb[None, :, 2]
    ty = ys[:, None] + eb[None, :, 1]
    tx = (xs[:, None] + eb[None, :, 0]) % NX
    wall = (tz < 0) | (tz >= NZ) | (ty < 0) | (ty >= NY)
    tz = np.where(wall, zs[:, None], tz)
    ty = np.where(wall, ys[:, None], ty)
    tx = np.where(wall, xs[:, None], tx)
    comp = np.where(wall, opp[None, :], np.arange(27)[None, :])
    idx = torch.from_numpy(np.stack([comp.ravel(), tz.ravel(), ty.ravel(), tx.ravel()])).cuda()
    mu = lam32[idx[0], idx[1], idx[2], idx[3]].reshape(len(zs), 27).cpu()
    fy = _gather_nodes(f0, zs, ys, xs).clone().requires_grad_(True)
    if field:
        force = _gather_nodes(ffield, zs, ys, xs).to(DT).requires_grad_(True)
    else:
        force = torch.tensor([FORCE] * len(zs), dtype=DT)
    ft = C.collide(fy, force, p)
    if field:
        want, want_gF = torch.autograd.grad(ft, (fy, force), grad_outputs=mu)
        got_gF = _gather_nodes(gfield, zs, ys, xs).to(DT)
        errF = (got_gF - want_gF).abs().max().item() / want_gF.abs().max().item()
        _say(f"force-field gradient at the sampled nodes: rel max err {errF:.2e}")
        assert errF < 2e-6
    else:
        (want,) = torch.autograd.grad(ft, (fy,), grad_outputs=mu)
    err = (got - want).abs().max().item() / want.abs().max().item()
    nwall = int(wall.any(1).sum())
    _say(f"512x512x160 duct adjoint, {storage} state{' + force field' if field else ''} (adjoint arrays {27 * lat.h.stride * 4 / 2**30:.2f} GiB), "
         f"{len(zs)} sampled nodes ({nwall} next to a wall): rel max err {err:.2e}")
    assert nwall >= 24
    assert err < 2e-6
