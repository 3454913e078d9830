"""GPU parity of the forward path (init, import/export, step, observables)
against the FP64 oracle, through the C ABI.

Tolerances (derived in the design notes): one FP32 step on FP32-rounded
inputs agrees element by element within 2e-7 absolute on populations of
magnitude <= 0.6; the 200-step Taylor-Green run on the 32x32x16 cuboid
grid must agree in velocity within 1e-5 relative L2.
"""

import math
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
    # name, grid, r, s, bc_y, bc_z, corr, force kind
    ("periodic_tiles_ragged", (300, 6, 5), 1.0, 0.5, "periodic", "periodic", "local", "none"),
    ("duct_walls_force_field", (37, 12, 10), 1.0, 0.25, "bounceback", "bounceback", "local", "field"),
    ("aniso_lowmach_uniform", (20, 9, 14), 0.5, 0.25, "periodic", "bounceback", "lowmach", "uniform"),
    ("off_walls_y", (24, 8, 6), 0.7, 1.3, "bounceback", "periodic", "off", "uniform"),
    ("single_node_axes", (1, 1, 1), 1.0, 0.5, "periodic", "periodic", "local", "field"),
]


@pytest.mark.parametrize("case", CASES, ids=[c[0] for c in CASES])
def test_single_step_matches_oracle(case):
    name, (nx, ny, nz), r, s, by, bz, corr, fkind = case
    _say("case", name)
    p = oracle.Params(nx, ny, nz, r=r, s=s, omega_nu=1.45, omega_xi=1.27, corr=corr, bc_y=by, bc_z=bz)
    f0 = fp32_rounded_state(random_state(p, 11), p)
    g = np.random.Generator(np.random.PCG64(12))
    uniform = (2e-5, -1e-5, 3e-6) if fkind == "uniform" else (0.0, 0.0, 0.0)
    field = torch.tensor(1e-4 * g.standard_normal((3, *p.shape))).to(torch.float32) if fkind == "field" else None
    lat = gpu_lattice(p, force=uniform)
    a, b = lat.new_state(), lat.new_state()
    lat.import_populations(a, f0.cuda())
    cur, _ = lat.step(a, b, 1, force=None if field is None else field.cuda().contiguous())
    got = lat.export_populations(cur).cpu()
    oforce = field.to(DT) if field is not None else uniform
    want = OL.step(f0, p, force=oforce)
    err = (got - want).abs().max().item()
    _say(f"{name}: max |f_gpu - f_oracle| = {err:.3e}")
    assert err < 2e-7


def test_import_export_roundtrip():
    p = oracle.Params(17, 5, 9, r=0.8, s=0.5, bc_y="bounceback", bc_z="periodic")
    f0 = fp32_rounded_state(random_state(p, 3), p)
    lat = gpu_lattice(p)
    st = lat.new_state()
    lat.import_populations(st, f0.cuda())
    back = lat.export_populations(st).cpu()
    assert (back - f0).abs().max().item() < 1e-15


def test_init_matches_oracle_equilibrium():
    w = W.TAYLOR_GREEN_32
    p = oracle_params(w)
    u = torch.tensor(W.initial_velocity(w))
    rho = torch.tensor(1.0 + 0.01 * W.gaussian_field(p.shape, 1.0, 5))
    lat = gpu_lattice(p)
    st = lat.new_state()
    lat.init(st, rho=rho, u=u)
    got = lat.export_populations(st).cpu()
    want = OL.init_equilibrium(rho, u, p)
    err = (got - want).abs().max().item()
    _say(f"init: max abs err {err:.3e}")
    assert err < 1e-9


def test_moments_match_oracle():
    p = oracle.Params(33, 10, 7, r=1.0, s=0.5, omega_nu=1.3, omega_xi=1.1, bc_y="bounceback")
    f0 = fp32_rounded_state(random_state(p, 5), p)
    g = np.random.Generator(np.random.PCG64(6))
    field = torch.tensor(1e-4 * g.standard_normal((3, *p.shape))).to(torch.float32)
    lat = gpu_lattice(p)
    st = lat.new_state()
    lat.import_populations(st, f0.cuda())
    m = lat.moments(st, force=field.cuda())
    rho, u = OL.observables(f0, p, force=field.to(DT))
    sums = OL.sums(f0, p, force=field.to(DT))
    assert (m.rho.cpu().to(DT) - rho).abs().max() < 2e-7
    assert (m.u.cpu().to(DT) - u).abs().max() < 2e-8
    got = m.sums.cpu()
    _say("sums gpu", got.tolist(), "oracle", sums.tolist())
    # totals are FP64 sums of the stored FP32 values: exact up to FP64 rounding
    assert abs(got[0] - sums[0]) / sums[0] < 1e-14
    assert torch.allclose(got[1:4], sums[1:4], rtol=1e-12, atol=1e-13)
    assert abs(got[4] - sums[4]) / sums[4] < 1e-12


def _taylor_green_run(storage, steps):
    w = W.TAYLOR_GREEN_32
    p = oracle_params(w)
    u0 = torch.tensor(W.initial_velocity(w))
    noise = torch.tensor(W.uniform_noise((27, *p.shape), w.extra["noise"], w.extra["noise_seed"]))
    lat = gpu_lattice(p, storage=storage)
    a, b = lat.new_state(), lat.new_state()
    lat.init(a, u=u0, perturb=noise)
    cur, _ = lat.step(a, b, steps)
    m = lat.moments(cur)
    torch.cuda.synchronize()
    return p, u0, noise, m


@pytest.fixture(scope="module")
def taylor_green_oracle():
    w = W.TAYLOR_GREEN_32
    p = oracle_params(w)
    u0 = torch.tensor(W.initial_velocity(w))
    noise = torch.tensor(W.uniform_noise((27, *p.shape), w.extra["noise"], w.extra["noise_seed"]))
    f = OL.init_equilibrium(torch.ones(p.shape, dtype=DT), u0, p) + noise
    f = OL.run(f, p, w.steps)
    rho, u = OL.observables(f, p)
    return rho, u, OL.sums(f, p)


def test_taylor_green_fp32_within_1e5(taylor_green_oracle):
    """Accuracy gate: FP32 GPU vs FP64 oracle, relative L2 of u after 200 steps <= 1e-5."""
    rho_o, u_o, sums_o = taylor_green_oracle
    _, _, _, m = _taylor_green_run("f32", W.TAYLOR_GREEN_32.steps)
    err = rel_l2(m.u.cpu(), u_o)
    err_rho = (m.rho.cpu().to(DT) - rho_o).abs().max().item()
    _say(f"taylor-green 200 steps FP32: rel L2(u) = {err:.3e}, max|drho| = {err_rho:.3e}")
    assert err <= 1e-5
    assert abs(m.sums[0].item() - sums_o[0].item()) / sums_o[0].item() < 1e-10


@pytest.mark.parametrize("storage,bound", [("f16", 2e-3), ("bf16", 3e-2), ("bf16_sr", 3e-2)])
def test_taylor_green_reduced_storage_error(taylor_green_oracle, storage, bound):
    """16-bit deviation storage: error against the FP64 oracle is stated, with a loose bound."""
    rho_o, u_o, sums_o = taylor_green_oracle
    _, _, _, m = _taylor_green_run(storage, W.TAYLOR_GREEN_32.steps)
    err = rel_l2(m.u.cpu(), u_o)
    e_err = abs(m.sums[4].item() - sums_o[4].item()) / sums_o[4].item()
    _say(f"taylor-green 200 steps {storage}: rel L2(u) = {err:.3e}, rel energy err = {e_err:.3e}")
    assert err <= bound


def test_duct_replica_matches_oracle():
    """Duct physics of the 64x128x32 workload on a 40x24x12 replica, 100 steps, uniform force."""
    w = W.DUCT_64
    p = oracle_params(w, nx=40, ny=24, nz=12)
    a_half, b_half = p.ny * p.r / 2, p.nz * p.s / 2
    fx = oracle.analytic.duct_force_for_centre_velocity(w.extra["u_centre"], a_half, b_half, 1.0, w.nu)
    force = (fx, 0.0, 0.0)
    lat = gpu_lattice(p, force=force)
    a, b = lat.new_state(), lat.new_state()
    lat.init(a)
    cur, _ = lat.step(a, b, 100)
    m = lat.moments(cur)
    f = OL.init_equilibrium(torch.ones(p.shape, dtype=DT), torch.zeros(3, *p.shape, dtype=DT), p)
    f = OL.run(f, p, 100, force=force)
    _, u = OL.observables(f, p, force=force)
    err = rel_l2(m.u.cpu(), u)
    _say(f"duct replica 100 steps: rel L2(u) = {err:.3e}")
    assert err <= 1e-5


def test_nonfinite_totals_are_reported():
    """A NaN population makes lbm_check_sums return LBM_ENONFINITE (failure detection)."""
    from paper_2107_14774_amd import _lib
    import paper_2107_14774_amd as P
    p = oracle.Params(8, 6, 4)
    f0 = fp32_rounded_state(random_state(p, 9), p)
    f0[3, 1, 2, 3] = float("nan")
    lat = gpu_lattice(p)
    st = lat.new_state()
    lat.import_populations(st, f0.cuda())
    m = lat.moments(st)
    with pytest.raises(_lib.LbmError) as e:
        P.lbm_check_sums(m.sums)
    assert e.value.code == _lib.LBM_ENONFINITE


def test_zero_steps_leave_the_state_unchanged():
    """nsteps = 0 is a valid call that launches nothing: two-buffer, AA, full corrections, forcing."""
    import paper_2107_14774_amd as P
    p = oracle.Params(12, 8, 6, r=1.0, s=0.5, bc_y="bounceback")
    f0 = fp32_rounded_state(random_state(p, 11), p)
    for layout in ("ab", "aa"):
        lat = P.Lattice(p.nx, p.ny, p.nz, r=p.r, s=p.s, cs2=p.cs2, omega_nu=p.omega_nu, omega_xi=p.omega_xi,
                        bc_y=p.bc_y, layout=layout)
        a = lat.new_state()
        b = None if layout == "aa" else lat.new_state()
        lat.import_populations(a, f0.cuda())
        before = lat.export_populations(a)
        cur, _ = lat.step(a, b, 0)
        assert cur is a and torch.equal(lat.export_populations(cur), before)
        cur, _ = lat.step_forcing(a, b, np.zeros((0, 3)))
        assert cur is a and torch.equal(lat.export_populations(cur), before)
    full = gpu_lattice(oracle.Params(12, 8, 6, r=1.0, s=0.5, corr="full"))
    a, b = full.new_state(), full.new_state()
    full.import_populations(a, f0.cuda())
    before = full.export_populations(a)
    da = full.density(a)
    cur, _, d_cur, _ = full.step_full(a, b, 0, da, full.field(1), "lagged")
    assert cur is a and d_cur is da and torch.equal(full.export_populations(cur), before)


@pytest.mark.parametrize("layout", ["ab", "aa"])
def test_lds_reservation_does_not_change_results(layout):
    """The FP32 one-node steps reserve LDS only to limit the blocks per CU (LBM_STEP_LDS, read when a
    handle is created): states with and without the reservation agree bit for bit, walls included."""
    import os
    import paper_2107_14774_amd as P
    p = oracle.Params(70, 9, 6, r=1.0, s=0.5, bc_z="bounceback" if layout == "ab" else "periodic")
    f0 = fp32_rounded_state(random_state(p, 17), p)
    out = []
    old = os.environ.get("LBM_STEP_LDS")
    try:
        for lds in ("0", None):
            if lds is None:
                os.environ.pop("LBM_STEP_LDS", None)
            else:
                os.environ["LBM_STEP_LDS"] = lds
            lat = P.Lattice(p.nx, p.ny, p.nz, r=p.r, s=p.s, cs2=p.cs2, omega_nu=p.omega_nu, omega_xi=p.omega_xi,
                            bc_z=p.bc_z, force=(1e-5, 0.0, -2e-6), layout=layout)
            a = lat.new_state()
            b = None if layout == "aa" else lat.new_state()
            lat.import_populations(a, f0.cuda())
            cur, _ = lat.step(a, b, 4)
            out.append(lat.export_populations(cur))
    finally:
        if old is None:
            os.environ.pop("LBM_STEP_LDS", None)
        else:
            os.environ["LBM_STEP_LDS"] = old
    print(f"{layout}: max |lds 0 - default| = {(out[0] - out[1]).abs().max().item():.3e}", flush=True)
    assert torch.equal(out[0], out[1])
