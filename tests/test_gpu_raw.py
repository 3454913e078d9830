"""GPU parity of the raw-moment scheme (Sec. 7) against the FP64 oracle, through the C ABI."""

import sys

import numpy as np
import pytest
import torch

import oracle
from oracle import lbm as OL
import workloads as W
from helpers import fp32_rounded_state, gpu_lattice, oracle_params, random_state, rel_l2

pytestmark = pytest.mark.gpu
DT = torch.float64


def _say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


CASES = [
    # name, grid, r, s, (bc_x, bc_y, bc_z), corr, force kind, lid
    ("periodic_ragged_local", (300, 6, 5), 1.0, 0.5, ("periodic",) * 3, "local", "none", None),
    ("duct_force_field_lowmach", (37, 12, 10), 1.0, 0.25, ("periodic", "bounceback", "bounceback"), "lowmach", "field", None),
    ("cavity_lid_off", (12, 16, 12), 0.75, 1.0, ("bounceback",) * 3, "off", "none", (0.06, 0.0, 0.0)),
    ("cavity_lid_full", (10, 12, 9), 0.5, 1.0, ("bounceback",) * 3, "full", "uniform", (0.05, 0.0, 0.02)),
]


@pytest.mark.parametrize("case", CASES, ids=[c[0] for c in CASES])
def test_raw_step_matches_oracle(case):
    name, (nx, ny, nz), r, s, (bx, by, bz), corr, fkind, lid = case
    _say("case", name)
    wv = ((0, 0, 0),) * 3 + ((lid or (0, 0, 0)),) + ((0, 0, 0),) * 2
    p = oracle.Params(nx, ny, nz, r=r, s=s, omega_nu=1.6, omega_xi=1.0, corr=corr, bc_x=bx, bc_y=by, bc_z=bz,
                      wall_velocity=wv, moments="raw")
    f0 = fp32_rounded_state(random_state(p, 19), p)
    g = np.random.Generator(np.random.PCG64(20))
    uniform = (2e-5, -1e-5, 3e-6) if fkind == "uniform" else (0.0, 0.0, 0.0)
    field = torch.tensor(1e-4 * g.standard_normal((3, *p.shape))).to(torch.float32) if fkind == "field" else None
    lat = gpu_lattice(p, force=uniform)
    a, b = lat.new_state(), lat.new_state()
    lat.import_populations(a, f0.cuda())
    fd = None if field is None else field.cuda().contiguous()
    if corr == "full":
        cur, _, _, _ = lat.step_full(a, b, 1, lat.field(1), None, "exact", force=fd)
    else:
        cur, _ = lat.step(a, b, 1, force=fd)
    got = lat.export_populations(cur).cpu()
    oforce = field.to(DT) if field is not None else uniform
    want = OL.step(f0, p, force=oforce)
    pc = oracle.Params(nx, ny, nz, r=r, s=s, omega_nu=1.6, omega_xi=1.0, corr=corr, bc_x=bx, bc_y=by, bc_z=bz,
                       wall_velocity=wv)
    effect = (OL.step(f0, pc, force=oforce) - want).abs().max().item()
    err = (got - want).abs().max().item()
    _say(f"{name}: max |f_gpu - f_oracle| = {err:.3e} (raw vs central differ by {effect:.3e})")
    assert err < 2e-7
    assert effect > 50 * err


def test_raw_taylor_green_run_matches_oracle():
    """200 steps of the 32x32x16 Taylor-Green workload with the raw-moment scheme."""
    w = W.TAYLOR_GREEN_32
    p0 = oracle_params(w)
    p = oracle.Params(p0.nx, p0.ny, p0.nz, r=p0.r, s=p0.s, cs2=p0.cs2, omega_nu=p0.omega_nu,
                      omega_xi=p0.omega_xi, corr="local", moments="raw")
    u0 = torch.tensor(W.initial_velocity(w))
    noise = torch.tensor(W.uniform_noise((27, *p.shape), w.extra["noise"], w.extra["noise_seed"]))
    lat = gpu_lattice(p)
    a, b = lat.new_state(), lat.new_state()
    lat.init(a, u=u0, perturb=noise)
    cur, _ = lat.step(a, b, w.steps)
    m = lat.moments(cur)
    f = OL.init_equilibrium(torch.ones(p.shape, dtype=DT), u0, p) + noise
    f = OL.run(f, p, w.steps)
    _, u = OL.observables(f, p)
    err = rel_l2(m.u.cpu(), u)
    _say(f"raw taylor-green 200 steps FP32: rel L2(u) = {err:.3e}")
    assert err <= 1e-5
