"""GPU parity of the full corrections (density-gradient terms of App. D)
against the FP64 oracle, through the C ABI: lbm_density, lbm_step_full in
its exact and lagged modes."""

import math
import sys

import numpy as np
import pytest
import torch

import oracle
from oracle import lbm as OL
import paper_2107_14774_amd as P
import workloads as W
from helpers import fp32_rounded_state, gpu_lattice, oracle_params, random_state, rel_l2

pytestmark = pytest.mark.gpu
DT = torch.float64


def _say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


CASES = [
    # name, grid, r, s, bc_y, bc_z, force kind
    ("periodic_tiles_ragged", (300, 6, 5), 1.0, 0.5, "periodic", "periodic", "none"),
    ("duct_walls_force_field", (37, 12, 10), 1.0, 0.25, "bounceback", "bounceback", "field"),
    ("aniso_walls_z", (20, 9, 14), 0.5, 0.25, "periodic", "bounceback", "uniform"),
    ("two_node_walls", (5, 2, 3), 1.3, 0.8, "bounceback", "periodic", "none"),
    ("single_node_axes", (1, 1, 1), 1.0, 0.5, "periodic", "periodic", "field"),
    # 192-wide blocks, three per row, the last one ragged; 256-wide blocks that fill the row
    ("blocks_192_ragged", (520, 3, 4), 1.0, 0.5, "bounceback", "periodic", "none"),
    ("blocks_256_full", (256, 4, 3), 0.5, 0.25, "periodic", "periodic", "uniform"),
]


@pytest.mark.parametrize("case", CASES, ids=[c[0] for c in CASES])
def test_full_single_step_matches_oracle(case):
    """One exact-mode step (gradient from the step's own input density) on random states."""
    name, (nx, ny, nz), r, s, by, bz, fkind = case
    _say("case", name)
    p = oracle.Params(nx, ny, nz, r=r, s=s, omega_nu=1.45, omega_xi=1.27, corr="full", bc_y=by, bc_z=bz)
    # Mach 0.1 as in the local-correction test: near Mach 1 the strain-rate system of App. D
    # becomes singular (C_sz -> 0) and amplifies rounding, on every precision
    f0 = fp32_rounded_state(random_state(p, 13), p)
    g = np.random.Generator(np.random.PCG64(14))
    uniform = (2e-5, -1e-5, 3e-6) if fkind == "uniform" else (0.0, 0.0, 0.0)
    field = torch.tensor(1e-4 * g.standard_normal((3, *p.shape))).to(torch.float32) if fkind == "field" else None
    lat = gpu_lattice(p, force=uniform)
    a, b = lat.new_state(), lat.new_state()
    lat.import_populations(a, f0.cuda())
    drho = lat.field(1)
    cur, _, _, _ = lat.step_full(a, b, 1, drho, None, "exact",
                                 force=None if field is None else field.cuda().contiguous())
    got = lat.export_populations(cur).cpu()
    oforce = field.to(DT) if field is not None else uniform
    want = OL.step(f0, p, force=oforce)
    err = (got - want).abs().max().item()
    # the density-gradient terms change this step by a visible amount (they are tested, not zero)
    p_loc = oracle.Params(nx, ny, nz, r=r, s=s, omega_nu=1.45, omega_xi=1.27, corr="local", bc_y=by, bc_z=bz)
    effect = (OL.step(f0, p_loc, force=oforce) - want).abs().max().item()
    _say(f"{name}: max |f_gpu - f_oracle| = {err:.3e} (size of the lambda terms {effect:.3e})")
    assert err < 2e-7
    if nx * ny * nz > 1:
        assert effect > 50 * err


def test_density_matches_oracle_and_the_step():
    p = oracle.Params(40, 7, 9, r=1.0, s=0.5, omega_nu=1.3, omega_xi=1.1, corr="full", bc_z="bounceback")
    f0 = fp32_rounded_state(random_state(p, 15), p)
    lat = gpu_lattice(p)
    a, b = lat.new_state(), lat.new_state()
    lat.import_populations(a, f0.cuda())
    d = lat.density(a)
    want = f0.sum(0) - 1.0
    err = (d.cpu().to(DT) - want).abs().max().item()
    _say(f"lbm_density: max abs err {err:.3e}")
    assert err < 1e-7
    # the lagged step writes the density of its own input state: bit-identical to lbm_density
    d_in = d.clone()
    d_out = torch.full_like(d, float("nan"))
    P.lbm_step_full(lat.h, 1, a, b, d_in, d_out, "lagged")
    assert torch.equal(d_out, d)


def _smooth_flow(p, carrier=0.05):
    """Taylor-Green vortex plus a density wave, carried along x and y (the lambda terms need u . grad rho)."""
    z, y, x = torch.meshgrid(torch.arange(p.nz, dtype=DT) * p.s, torch.arange(p.ny, dtype=DT) * p.r,
                             torch.arange(p.nx, dtype=DT), indexing="ij")
    Lx, Ly, Lz = p.nx, p.ny * p.r, p.nz * p.s
    kx, ky, kz = 2 * math.pi / Lx, 2 * math.pi / Ly, 2 * math.pi / Lz
    u = torch.zeros(3, *p.shape, dtype=DT)
    u[0] = 0.03 * torch.sin(kx * x) * torch.cos(ky * y) * torch.cos(kz * z) + carrier
    u[1] = -0.03 * (kx / ky) * torch.cos(kx * x) * torch.sin(ky * y) * torch.cos(kz * z) + 0.5 * carrier
    rho = 1.0 + 0.01 * torch.cos(kx * x + ky * y) + 0.005 * torch.sin(kz * z)
    return rho, u


@pytest.fixture(scope="module")
def full_runs():
    p = oracle_params(W.TAYLOR_GREEN_32, corr="full")
    rho, u = _smooth_flow(p)
    f = fp32_rounded_state(OL.init_equilibrium(rho, u, p), p)
    steps = 100
    fe = OL.run(f, p, steps, lagged=False)
    fl = OL.run(f, p, steps, lagged=True)
    p_loc = oracle_params(W.TAYLOR_GREEN_32, corr="local")
    floc = OL.run(f, p_loc, steps)
    return p, f, steps, {m: OL.observables(x, p)[1] for m, x in (("exact", fe), ("lagged", fl), ("local", floc))}


@pytest.mark.parametrize("mode", ["exact", "lagged"])
def test_full_run_matches_oracle(full_runs, mode):
    """100 steps on the 32x32x16 cuboid grid (r = 1, s = 1/2) of a carried vortex with a density wave."""
    p, f0, steps, u_o = full_runs
    lat = gpu_lattice(p)
    a, b = lat.new_state(), lat.new_state()
    lat.import_populations(a, f0.cuda())
    da, db = lat.density(a), lat.field(1)
    cur, _, _, _ = lat.step_full(a, b, steps, da, db, mode)
    u = lat.moments(cur).u.cpu()
    carrier = torch.tensor([0.05, 0.025, 0.0], dtype=DT)[:, None, None, None]
    err = rel_l2(u.to(DT) - carrier, u_o[mode] - carrier)
    other = "lagged" if mode == "exact" else "exact"
    d_modes = rel_l2(u_o[other] - carrier, u_o[mode] - carrier)
    d_local = rel_l2(u_o["local"] - carrier, u_o[mode] - carrier)
    _say(f"full {mode}, {steps} steps: rel L2(u - U) vs oracle {err:.3e}; "
         f"oracle {other} differs by {d_modes:.3e}, local by {d_local:.3e}")
    assert err <= 1e-5
    assert d_local > 100 * err


def test_lagged_run_split_over_calls_equals_one_call():
    p = oracle.Params(48, 10, 8, r=1.0, s=0.5, omega_nu=1.4, omega_xi=1.2, corr="full", bc_y="bounceback")
    rho, u = _smooth_flow(p)
    lat = gpu_lattice(p)
    a, b = lat.new_state(), lat.new_state()
    lat.init(a, rho=rho, u=u)
    a2, b2 = lat.new_state(), lat.new_state()
    a2.copy_(a)
    da, db = lat.density(a), lat.field(1)
    cur, _, _, _ = lat.step_full(a, b, 11, da, db, "lagged")
    one = lat.export_populations(cur)
    da2, db2 = lat.density(a2), lat.field(1)
    cur2, scr2, d_cur, d_oth = lat.step_full(a2, b2, 4, da2, db2, "lagged")
    cur2, _, _, _ = lat.step_full(cur2, scr2, 7, d_cur, d_oth, "lagged")
    assert torch.equal(lat.export_populations(cur2), one)


def test_full_f16_storage_tracks_oracle(full_runs):
    """16-bit deviation storage: the full path adds no error beyond that of the storage format,
    measured as the local-correction path's FP16 error on the same flow against its own oracle run."""
    p, f0, steps, u_o = full_runs
    carrier = torch.tensor([0.05, 0.025, 0.0], dtype=DT)[:, None, None, None]
    errs = {}
    for corr in ("full", "local"):
        pc = oracle_params(W.TAYLOR_GREEN_32, corr=corr)
        lat = gpu_lattice(pc, storage="f16")
        a, b = lat.new_state(), lat.new_state()
        lat.import_populations(a, f0.cuda())
        if corr == "full":
            da, db = lat.density(a), lat.field(1)
            cur, _, _, _ = lat.step_full(a, b, steps, da, db, "lagged")
            ref = u_o["lagged"]
        else:
            cur, _ = lat.step(a, b, steps)
            ref = u_o["local"]
        u = lat.moments(cur).u.cpu()
        errs[corr] = rel_l2(u.to(DT) - carrier, ref - carrier)
    _say(f"f16, {steps} steps: rel L2(u - U) vs oracle: full {errs['full']:.3e}, local {errs['local']:.3e}")
    assert errs["full"] <= 5e-3
    assert errs["full"] <= 1.2 * errs["local"]
