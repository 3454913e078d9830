"""GPU parity of the three gather paths on every grid and of grids beyond 2^30 nodes.

lbm_create picks the row-addressed path for periodic grids (any size), 32-bit
offsets across the state for walled states below 4 GiB, and 64-bit slots for
larger walled states.  The testing override LBM_GATHER_KIND=1 or 2 makes small
grids take the more general paths, so the cases below run each path (forward
step, adjoint step) against the FP64 oracle at sizes the oracle handles.  The
last test runs a periodic FP16 grid of 1024^3 = 2^30 nodes with a force field
in the production launch and checks sampled nodes (lbm_export_nodes) against
the oracle, which collides the upstream neighbours of each sampled node.
"""

import contextlib
import os
import sys

import numpy as np
import pytest
import torch

import oracle
from oracle import collision as C
from oracle import equilibrium as EQ
from oracle import gradient as G
from oracle import lattice as LT
from oracle import lbm as OL
import paper_2107_14774_amd as P
from helpers import fp32_rounded_state, gpu_lattice, random_state

pytestmark = pytest.mark.gpu
DT = torch.float64


def _say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


@contextlib.contextmanager
def _kind(kind):
    """LBM_GATHER_KIND is read when a handle is created."""
    old = os.environ.get("LBM_GATHER_KIND")
    os.environ["LBM_GATHER_KIND"] = str(kind)
    try:
        yield
    finally:
        if old is None:
            del os.environ["LBM_GATHER_KIND"]
        else:
            os.environ["LBM_GATHER_KIND"] = old


CASES = [
    # name, grid, r, s, (bc_x, bc_y, bc_z), moving faces, storage
    ("periodic_ragged_field", (300, 6, 5), 1.0, 0.5, ("periodic",) * 3, None, "f32"),
    ("duct_y_walls_z_periodic", (37, 12, 10), 1.0, 0.25, ("periodic", "bounceback", "periodic"), None, "f32"),
    ("box_moving_faces", (14, 10, 8), 0.5, 1.0, ("bounceback",) * 3,
     ((0, 0, 0), (0, 0.01, 0), (0, 0, 0), (0.05, 0, 0.02), (0.03, 0, 0), (0, 0, 0)), "f32"),
    ("periodic_f16_field", (70, 9, 6), 0.5, 0.25, ("periodic",) * 3, None, "f16"),
]


@pytest.mark.parametrize("kind", [1, 2])
@pytest.mark.parametrize("case", CASES, ids=[c[0] for c in CASES])
def test_forced_gather_kind_step_matches_oracle(case, kind):
    name, (nx, ny, nz), r, s, (bx, by, bz), wv, storage = case
    _say("case", name, "gather kind", kind)
    p = oracle.Params(nx, ny, nz, r=r, s=s, omega_nu=1.45, omega_xi=1.27, corr="local", bc_x=bx, bc_y=by, bc_z=bz,
                      wall_velocity=wv or ((0, 0, 0),) * 6)
    f0 = fp32_rounded_state(random_state(p, 13), p)
    g = np.random.Generator(np.random.PCG64(14))
    field = torch.tensor(1e-4 * g.standard_normal((3, *p.shape))).to(torch.float32)
    with _kind(kind):
        lat = gpu_lattice(p, storage=storage)
    a, b = lat.new_state(), lat.new_state()
    lat.import_populations(a, f0.cuda())
    start = lat.export_populations(a).cpu()               # the stored (storage-rounded) start
    cur, _ = lat.step(a, b, 1, force=field.cuda().contiguous())
    got = lat.export_populations(cur).cpu()
    want = OL.step(start, p, force=field.to(DT))
    err = (got - want).abs().max().item()
    dev = (want - EQ.rest_weights(p.r, p.s, p.cs2)[:, None, None, None]).abs().max().item()
    _say(f"{name}, kind {kind}: max |f_gpu - f_oracle| = {err:.3e} (max deviation {dev:.2e})")
    assert err < (2e-7 if storage == "f32" else 2e-3 * dev)


@pytest.mark.parametrize("kind", [1, 2])
@pytest.mark.parametrize("bcs", [("periodic",) * 3, ("bounceback", "bounceback", "periodic")],
                         ids=["periodic", "walls_xy"])
def test_forced_gather_kind_adjoint_matches_oracle(bcs, kind):
    p = oracle.Params(19, 10, 8, r=1.0, s=0.5, omega_nu=1.45, omega_xi=1.27, corr="local", bc_x=bcs[0], bc_y=bcs[1],
                      bc_z=bcs[2])
    f0 = fp32_rounded_state(random_state(p, 21), p)
    g = np.random.Generator(np.random.PCG64(22))
    force = torch.tensor(1e-4 * g.standard_normal((3, *p.shape))).to(torch.float32)
    lam_f = torch.tensor(g.standard_normal((27, *p.shape)))
    with _kind(kind):
        lat = gpu_lattice(p)
    st = lat.new_state()
    lat.import_populations(st, f0.cuda())
    lam_in, lam_out = lat.new_adjoint(), lat.new_adjoint()
    P.lbm_adjoint_from_natural(lat.h, lam_f.cuda(), lam_in)
    gF = torch.zeros((3, *p.shape), dtype=torch.float32, device="cuda")
    P.lbm_step_adjoint(lat.h, st, lam_in, lam_out, force.cuda(), gF)
    got = torch.empty((27, *p.shape), dtype=DT, device="cuda")
    P.lbm_adjoint_to_natural(lat.h, lam_out, got)
    want_f, want_F = G.step_vjp(f0, p, force.to(DT), lam_f)
    err = (got.cpu() - want_f).abs().max().item() / want_f.abs().max().item()
    errF = (gF.cpu().to(DT) - want_F).abs().max().item() / want_F.abs().max().item()
    _say(f"adjoint {bcs}, kind {kind}: rel max err lambda {err:.2e}, force grad {errF:.2e}")
    assert err < 2e-6 and errF < 2e-5


def test_export_nodes_equals_full_export():
    p = oracle.Params(130, 7, 5, r=1.0, s=0.5, bc_y="bounceback")
    lat = gpu_lattice(p, storage="f16")
    st = lat.new_state()
    lat.import_populations(st, random_state(p, 31).cuda())
    full = lat.export_populations(st)
    nodes = torch.tensor([0, 1, 129, 130, 2000, p.n - 1, -1, p.n], dtype=torch.int64, device="cuda")
    f = torch.empty((27, nodes.numel()), dtype=DT, device="cuda")
    P.lbm_export_nodes(lat.h, st, nodes, f)
    flat = full.reshape(27, -1)
    assert torch.equal(f[:, :6], flat[:, nodes[:6]])
    assert torch.isnan(f[:, 6:]).all()                        # outside [0, n): NaN


def test_periodic_fp16_grid_of_2_30_nodes_with_force_field():
    """1024^3 nodes (2^30), FP16 storage (two 54 GiB states), periodic, per-node force field: one step
    in the production launch, 64 sampled nodes (faces, edges, corners and the last node among them)
    against the oracle."""
    n1 = 1024
    p = oracle.Params(n1, n1, n1, r=1.0, s=0.5, cs2=1.0 / 12.0, omega_nu=1.6, omega_xi=1.2, corr="local")
    lat = gpu_lattice(p, storage="f16")
    assert lat.n == 1 << 30 and lat.h.state_bytes == 27 * 2 * (1 << 30)
    dev_ = torch.device("cuda")
    ax = [torch.arange(n1, dtype=DT, device=dev_) * (2 * np.pi / n1) for _ in range(3)]
    X, Y, Z = ax[0][None, None, :], ax[1][None, :, None], ax[2][:, None, None]
    u = torch.empty((3, n1, n1, n1), dtype=DT, device=dev_)
    u[0] = 0.03 * torch.sin(X) * torch.cos(Y) * torch.cos(2 * Z)
    u[1] = -0.03 * torch.cos(X) * torch.sin(Y) * torch.cos(2 * Z)
    u[2] = 0.01 * torch.sin(3 * X + Y)

    def force_at(zz, yy, xx, xp):
        """The force field (FP64 formula, then FP32 like the field passed to the GPU)."""
        xs, ys, zs = (2 * np.pi / n1) * xx, (2 * np.pi / n1) * yy, (2 * np.pi / n1) * zz
        fx = 1e-5 * xp.sin(zs + ys) + 0.0 * xs
        fy = 1e-5 * xp.cos(xs - zs) + 0.0 * ys
        fz = 5e-6 * xp.sin(2 * xs) * xp.cos(ys)
        return fx, fy, fz

    force = torch.empty((3, n1, n1, n1), dtype=torch.float32, device=dev_)
    for c, comp in enumerate(force_at(torch.arange(n1, dtype=DT, device=dev_)[:, None, None],
                                      torch.arange(n1, dtype=DT, device=dev_)[None, :, None],
                                      torch.arange(n1, dtype=DT, device=dev_)[None, None, :], torch)):
        force[c] = comp.expand(n1, n1, n1).to(torch.float32)
    a, b = lat.new_state(), lat.new_state()
    lat.init(a, u=u)
    del u
    torch.cuda.synchronize()
    g = np.random.Generator(np.random.PCG64(101))
    pts = [(0, 0, 0), (n1 - 1, n1 - 1, n1 - 1), (0, n1 - 1, 17), (n1 - 1, 0, 1023), (512, 0, 0), (3, 700, n1 - 1)]
    pts += [tuple(int(v) for v in g.integers(0, n1, 3)) for _ in range(64 - len(pts))]
    zs, ys, xs = (np.array([q[i] for q in pts]) for i in range(3))
    samples = (zs * n1 + ys) * n1 + xs
    eb = LT.ebar().numpy()
    nb_z, nb_y, nb_x = ((zs[None, :] - eb[:, 2:3]) % n1, (ys[None, :] - eb[:, 1:2]) % n1, (xs[None, :] - eb[:, 0:1]) % n1)
    nb = ((nb_z * n1 + nb_y) * n1 + nb_x).ravel()                        # (27 * samples,), direction-major
    f_nb = torch.empty((27, nb.size), dtype=DT, device=dev_)
    P.lbm_export_nodes(lat.h, a, torch.from_numpy(nb).to(dev_), f_nb)
    cur, _ = lat.step(a, b, 1, force=force)
    del force
    f_gpu = torch.empty((27, samples.size), dtype=DT, device=dev_)
    P.lbm_export_nodes(lat.h, cur, torch.from_numpy(samples).to(dev_), f_gpu)
    f_gpu = f_gpu.cpu()
    # oracle: collide every upstream neighbour from the stored start and stream into the sampled node
    fx, fy, fz = force_at(nb_z.ravel().astype(np.float64), nb_y.ravel().astype(np.float64),
                          nb_x.ravel().astype(np.float64), np)
    F = torch.from_numpy(np.stack([fx, fy, fz], 1)).to(torch.float32).to(DT)
    ft = C.collide(f_nb.T.cpu(), F, p).reshape(27, samples.size, 27)
    want = torch.stack([ft[a_, :, a_] for a_ in range(27)])            # f_a(x) = f~_a(x - e_a)
    err = (f_gpu - want).abs().max().item()
    dev = (want - EQ.rest_weights(p.r, p.s, p.cs2)[:, None]).abs().max().item()
    _say(f"1024^3 FP16 with force field, one step, 64 sampled nodes: max |f_gpu - f_oracle| = {err:.3e} "
         f"(max deviation {dev:.2e})")
    assert err < 2e-3 * dev
    del a, b, cur, lat
    torch.cuda.empty_cache()
