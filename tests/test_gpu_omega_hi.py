"""GPU parity of the general higher-order rate (omega_hi != 1: every moment of
order >= 3 relaxes with it, App. D) against the FP64 oracle, through the C ABI:
single steps over boundaries, corrections and both moment bases, a 200-step
Taylor-Green run in FP32 and FP16 storage, and the adjoint step."""

import sys

import numpy as np
import pytest
import torch

import oracle
from oracle import gradient as G
from oracle import lbm as OL
import workloads as W
import paper_2107_14774_amd as P
from helpers import fp32_rounded_state, gpu_lattice, oracle_params, random_state, rel_l2

pytestmark = pytest.mark.gpu
DT = torch.float64
NO_WALLS = ((0, 0, 0),) * 6


def _say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def _params(grid, r, s, bcs, corr, moments, omega_hi, wv=NO_WALLS):
    nx, ny, nz = grid
    bx, by, bz = bcs
    return oracle.Params(nx, ny, nz, r=r, s=s, omega_nu=1.55, omega_xi=1.1, omega_hi=omega_hi, corr=corr,
                         bc_x=bx, bc_y=by, bc_z=bz, wall_velocity=wv, moments=moments)


LID = ((0, 0, 0),) * 3 + ((0.05, 0, 0.02),) + ((0, 0, 0),) * 2
CASES = [
    # name, grid, r, s, (bc_x, bc_y, bc_z), corr, moments, omega_hi, force kind, wall velocities
    ("periodic_ragged_local", (300, 6, 5), 1.0, 0.5, ("periodic",) * 3, "local", "central", 0.8, "uniform", NO_WALLS),
    ("duct_field_lowmach", (37, 12, 10), 1.0, 0.25, ("periodic", "bounceback", "bounceback"), "lowmach", "central",
     1.6, "field", NO_WALLS),
    ("cavity_lid_off_raw", (12, 16, 12), 0.75, 1.0, ("bounceback",) * 3, "off", "raw", 1.3, "none", LID),
    ("cavity_lid_full", (10, 12, 9), 0.5, 1.0, ("bounceback",) * 3, "full", "central", 0.6, "uniform", LID),
    ("periodic_raw_full_field", (70, 5, 4), 1.0, 0.5, ("periodic",) * 3, "full", "raw", 1.9, "field", NO_WALLS),
]


@pytest.mark.parametrize("case", CASES, ids=[c[0] for c in CASES])
def test_omega_hi_step_matches_oracle(case):
    name, grid, r, s, bcs, corr, moments, omega_hi, fkind, wv = case
    _say("case", name)
    p = _params(grid, r, s, bcs, corr, moments, omega_hi, wv)
    f0 = fp32_rounded_state(random_state(p, 51), p)
    g = np.random.Generator(np.random.PCG64(52))
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
    unit = _params(grid, r, s, bcs, corr, moments, 1.0, wv)
    effect = (OL.step(f0, unit, force=oforce) - want).abs().max().item()
    err = (got - want).abs().max().item()
    mass = abs(got.sum().item() - want.sum().item())
    _say(f"{name}: max |f_gpu - f_oracle| = {err:.3e} (omega_hi {omega_hi} vs 1 differ by {effect:.3e}), "
         f"mass diff {mass:.2e}")
    assert err < 2e-7
    assert effect > 50 * err
    assert mass < 1e-9 * p.nx * p.ny * p.nz


@pytest.fixture(scope="module")
def tg_oracle_omega_hi():
    """The 32x32x16 Taylor-Green workload with omega_hi = 1.5, 200 oracle steps."""
    w = W.TAYLOR_GREEN_32
    p0 = oracle_params(w)
    p = oracle.Params(p0.nx, p0.ny, p0.nz, r=p0.r, s=p0.s, cs2=p0.cs2, omega_nu=p0.omega_nu,
                      omega_xi=p0.omega_xi, omega_hi=1.5, corr="local")
    u0 = torch.tensor(W.initial_velocity(w))
    noise = torch.tensor(W.uniform_noise((27, *p.shape), w.extra["noise"], w.extra["noise_seed"]))
    f = OL.init_equilibrium(torch.ones(p.shape, dtype=DT), u0, p) + noise
    f = OL.run(f, p, w.steps)
    _, u = OL.observables(f, p)
    return w, p, u0, noise, u


@pytest.mark.parametrize("storage,bound", [("f32", 1e-5), ("f16", 2e-3)])
def test_omega_hi_taylor_green_run(tg_oracle_omega_hi, storage, bound):
    w, p, u0, noise, u_want = tg_oracle_omega_hi
    lat = gpu_lattice(p, storage=storage)
    a, b = lat.new_state(), lat.new_state()
    lat.init(a, u=u0, perturb=noise)
    cur, _ = lat.step(a, b, w.steps)
    m = lat.moments(cur)
    err = rel_l2(m.u.cpu(), u_want)
    _say(f"taylor-green 200 steps, omega_hi = 1.5, {storage}: rel L2(u) = {err:.3e}")
    assert err <= bound


ADJ_CASES = [
    ("periodic_ragged_local", (300, 5, 4), 1.0, 0.5, ("periodic",) * 3, "local", "central", 0.7, NO_WALLS),
    ("duct_raw_lowmach", (13, 9, 8), 0.5, 0.25, ("bounceback", "bounceback", "periodic"), "lowmach", "raw", 1.4,
     NO_WALLS),
    ("cavity_lid_off", (9, 8, 7), 0.5, 1.0, ("bounceback",) * 3, "off", "central", 1.8, LID),
]


@pytest.mark.parametrize("case", ADJ_CASES, ids=[c[0] for c in ADJ_CASES])
def test_omega_hi_adjoint_matches_oracle_vjp(case):
    name, grid, r, s, bcs, corr, moments, omega_hi, wv = case
    _say("case", name)
    p = _params(grid, r, s, bcs, corr, moments, omega_hi, wv)
    f0 = fp32_rounded_state(random_state(p, 53), p)
    g = np.random.Generator(np.random.PCG64(54))
    force = torch.tensor(1e-4 * g.standard_normal((3, *p.shape))).to(torch.float32)
    lam_f = torch.tensor(g.standard_normal((27, *p.shape)))
    lat = gpu_lattice(p)
    st = lat.new_state()
    lat.import_populations(st, f0.cuda())
    lam_in, lam_out = lat.new_adjoint(), lat.new_adjoint()
    P.lbm_adjoint_from_natural(lat.h, lam_f.cuda(), lam_in)
    gF = torch.zeros((3, *p.shape), dtype=torch.float32, device="cuda")
    gFu = torch.zeros(3, dtype=torch.float64, device="cuda")
    P.lbm_step_adjoint(lat.h, st, lam_in, lam_out, force.cuda(), gF, gFu)
    got = torch.empty((27, *p.shape), dtype=DT, device="cuda")
    P.lbm_adjoint_to_natural(lat.h, lam_out, got)
    want_f, want_F = G.step_vjp(f0, p, force.to(DT), lam_f)
    err = (got.cpu() - want_f).abs().max().item() / want_f.abs().max().item()
    errF = (gF.cpu().to(DT) - want_F).abs().max().item() / want_F.abs().max().item()
    unit_f, _ = G.step_vjp(f0, _params(grid, r, s, bcs, corr, moments, 1.0, wv), force.to(DT), lam_f)
    effect = (unit_f - want_f).abs().max().item() / want_f.abs().max().item()
    _say(f"{name}: rel max err lambda {err:.2e}, force grad {errF:.2e} (omega_hi effect {effect:.2e})")
    assert err < 2e-6
    assert errF < 2e-5
    assert effect > 100 * err
