"""GPU parity of the wall treatment against the FP64 oracle, through the C
ABI: halfway bounce-back on x, moving faces (momentum-augmented bounce-back,
Sec. 4 / eq. 69), edge and corner links, a shallow-cavity replica, and the
Couette fixed point."""

import sys

import numpy as np
import pytest
import torch

import oracle
from oracle import lbm as OL
from helpers import fp32_rounded_state, gpu_lattice, random_state, rel_l2

pytestmark = pytest.mark.gpu
DT = torch.float64
Z3 = (0.0, 0.0, 0.0)


def _say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def _walls(**faces):
    order = ("xm", "xp", "ym", "yp", "zm", "zp")
    return tuple(tuple(faces.get(f, Z3)) for f in order)


CASES = [
    # name, grid, r, s, (bc_x, bc_y, bc_z), wall velocities, corr
    ("cavity_lid_x", (14, 10, 8), 0.5, 1.0, ("bounceback",) * 3, _walls(yp=(0.05, 0, 0)), "local"),
    ("cavity_two_moving_faces", (12, 9, 10), 1.0, 0.5, ("bounceback",) * 3,
     _walls(yp=(0.04, 0, -0.02), zm=(0.03, 0.01, 0)), "local"),
    ("x_walls_moving_face", (9, 5, 6), 0.8, 0.6, ("bounceback", "periodic", "periodic"),
     _walls(xp=(0, 0.02, 0.03)), "lowmach"),
    ("x_walls_stationary_ragged", (70, 3, 4), 1.0, 0.5, ("bounceback", "periodic", "bounceback"), _walls(), "off"),
    ("cavity_full_corrections", (13, 8, 7), 0.5, 1.0, ("bounceback",) * 3, _walls(yp=(0.05, 0, 0)), "full"),
]


@pytest.mark.parametrize("case", CASES, ids=[c[0] for c in CASES])
def test_wall_step_matches_oracle(case):
    name, (nx, ny, nz), r, s, (bx, by, bz), wv, corr = case
    _say("case", name)
    p = oracle.Params(nx, ny, nz, r=r, s=s, omega_nu=1.4, omega_xi=1.25, corr=corr,
                      bc_x=bx, bc_y=by, bc_z=bz, wall_velocity=wv)
    f0 = fp32_rounded_state(random_state(p, 17), p)
    lat = gpu_lattice(p)
    a, b = lat.new_state(), lat.new_state()
    lat.import_populations(a, f0.cuda())
    if corr == "full":
        cur, _, _, _ = lat.step_full(a, b, 1, lat.field(1), None, "exact")
    else:
        cur, _ = lat.step(a, b, 1)
    got = lat.export_populations(cur).cpu()
    want = OL.step(f0, p)
    err = (got - want).abs().max().item()
    p_still = oracle.Params(nx, ny, nz, r=r, s=s, omega_nu=1.4, omega_xi=1.25, corr=corr, bc_x=bx, bc_y=by, bc_z=bz)
    effect = (OL.step(f0, p_still) - want).abs().max().item()
    _say(f"{name}: max |f_gpu - f_oracle| = {err:.3e} (size of the wall-velocity terms {effect:.3e})")
    assert err < 2e-7


def test_shallow_cavity_replica_matches_oracle():
    """The cuboid shallow cavity (L/H = 4, W/H = 2, r = 0.406, s = 1.3, cs2 = 0.04) at Ny = 16:
    26 x 16 x 10 nodes, lid along x, 300 steps from rest."""
    r, s, cs2 = 26 / 64, 1.3, 0.04
    U = 0.04
    nu = U * 26 * 4 / 64 * 16 / 100          # Re = U L / nu = 100 with L = 4 H, H = 16 r
    p = oracle.Params(26, 16, 10, r=r, s=s, cs2=cs2, omega_nu=1 / (nu / cs2 + 0.5), omega_xi=1 / (nu / cs2 + 0.5),
                      corr="local", bc_x="bounceback", bc_y="bounceback", bc_z="bounceback",
                      wall_velocity=_walls(yp=(U, 0, 0)))
    steps = 300
    lat = gpu_lattice(p)
    a, b = lat.new_state(), lat.new_state()
    lat.init(a)
    cur, _ = lat.step(a, b, steps)
    m = lat.moments(cur)
    f = OL.init_equilibrium(torch.ones(p.shape, dtype=DT), torch.zeros(3, *p.shape, dtype=DT), p)
    f = OL.run(f, p, steps)
    rho, u = OL.observables(f, p)
    err = rel_l2(m.u.cpu(), u)
    mass = m.sums[0].item()
    _say(f"shallow cavity replica {steps} steps: rel L2(u) = {err:.3e}, mass gpu {mass:.9f} oracle {rho.sum().item():.9f}")
    assert err <= 1e-5
    # the oracle keeps the mass exactly; FP32 rounding of the wall terms leaves about 1e-9
    assert abs(mass - rho.sum().item()) / rho.sum().item() < 5e-9


def test_couette_fixed_point_on_the_gpu():
    """Plane Couette flow on a cuboid grid (r = 1/2) started from the exact linear profile stays on it."""
    U, ny = 0.03, 24
    p = oracle.Params(4, ny, 3, r=0.5, s=1.0, omega_nu=1.2, omega_xi=1.2, bc_y="bounceback",
                      wall_velocity=_walls(yp=(U, 0, 0)))
    prof = U * (torch.arange(ny, dtype=DT) + 0.5) / ny
    u = torch.zeros(3, *p.shape, dtype=DT)
    u[0] = prof[None, :, None].expand(p.shape)
    lat = gpu_lattice(p)
    a, b = lat.new_state(), lat.new_state()
    lat.init(a, rho=torch.full(p.shape, 1.05, dtype=DT), u=u)
    cur, _ = lat.step(a, b, 3000)
    m = lat.moments(cur)
    err = (m.u.cpu().to(DT) - u).abs().max().item() / U
    _say(f"couette after 3000 steps: max |u - u_exact| / U = {err:.3e}")
    assert err < 1e-5
