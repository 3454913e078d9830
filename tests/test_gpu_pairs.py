"""GPU check of the 16-bit steps that run two x-adjacent nodes per thread
(periodic grids with even nx and unit higher-order rate, two-buffer and AA
layouts; a general higher-order rate runs the one-node kernels): they gather the same
values and run the same collision as the one-node kernels (selected with
LBM_PAIRS=0), so the states must agree bit for bit; and the two-buffer step
must match the FP64 oracle like the one-node kernel."""

import contextlib
import os
import sys

import numpy as np
import pytest
import torch

import oracle
from oracle import lbm as OL
from helpers import gpu_lattice, random_state

pytestmark = pytest.mark.gpu
DT = torch.float64


def _say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


@contextlib.contextmanager
def _pairs(enabled):
    """LBM_PAIRS is read when a handle is created."""
    old = os.environ.get("LBM_PAIRS")
    os.environ["LBM_PAIRS"] = "1" if enabled else "0"
    try:
        yield
    finally:
        if old is None:
            del os.environ["LBM_PAIRS"]
        else:
            os.environ["LBM_PAIRS"] = old


def _lattice(p, storage, force, pairs):
    with _pairs(pairs):
        return gpu_lattice(p, storage=storage, force=force)


CASES = [
    # name, grid, r, s, corr, moments, omega_hi, storage, force field
    ("ragged_local_f16", (300, 6, 5), 1.0, 0.5, "local", "central", 1.0, "f16", False),
    ("field_lowmach_bf16", (128, 9, 7), 0.5, 0.25, "lowmach", "central", 1.0, "bf16", True),
    ("raw_off_f16", (70, 8, 6), 1.0, 0.5, "off", "raw", 1.0, "f16", True),
    ("odd_words_f16", (130, 5, 4), 0.75, 1.0, "local", "central", 1.0, "f16", False),
    ("two_wide_bf16", (2, 7, 5), 1.0, 0.5, "local", "raw", 1.0, "bf16", True),
    ("stochastic_bf16sr", (300, 6, 5), 1.0, 0.5, "local", "central", 1.0, "bf16_sr", True),
]


@pytest.mark.parametrize("case", CASES, ids=[c[0] for c in CASES])
def test_pair_step_equals_one_node_step(case):
    name, (nx, ny, nz), r, s, corr, moments, omega_hi, storage, field = case
    _say("case", name)
    p = oracle.Params(nx, ny, nz, r=r, s=s, omega_nu=1.45, omega_xi=1.2, omega_hi=omega_hi, corr=corr,
                      moments=moments)
    f0 = random_state(p, 71)
    g = np.random.Generator(np.random.PCG64(72))
    force = torch.tensor(1e-4 * g.standard_normal((3, *p.shape))).to(torch.float32).cuda() if field else None
    uniform = (1e-5, -2e-6, 3e-6)
    one = _lattice(p, storage, uniform, pairs=False)
    two = _lattice(p, storage, uniform, pairs=True)
    a1, b1 = one.new_state(), one.new_state()
    a2, b2 = two.new_state(), two.new_state()
    one.import_populations(a1, f0.cuda())
    two.import_populations(a2, f0.cuda())
    start = two.export_populations(a2).cpu()
    for n in (1, 4):
        a1, b1 = one.step(a1, b1, n, force)
        a2, b2 = two.step(a2, b2, n, force)
        f1, f2 = one.export_populations(a1), two.export_populations(a2)
        _say(f"{name}: max |pairs - one node| = {(f1 - f2).abs().max().item():.3e}")
        assert torch.equal(f1, f2)
    # one step of the pair kernel against the oracle from the same (16-bit) start
    st, sb = two.new_state(), two.new_state()
    two.import_populations(st, start.cuda())
    cur, _ = two.step(st, sb, 1, force)
    got = two.export_populations(cur).cpu()
    want = OL.step(start, p, force=force.cpu().to(DT) if field else uniform)
    w = oracle.equilibrium.rest_weights(p.r, p.s, p.cs2)[:, None, None, None]
    err = (got - want).abs().max().item()
    dev = (want - w).abs().max().item()
    _say(f"{name}: one pair step vs FP64 oracle: max error {err:.2e} (max deviation {dev:.2e})")
    bound = 2e-3 if storage == "f16" else 1.6e-2       # 11 / 8 significand bits on the deviations
    assert err < bound * dev


AA_CASES = [
    ("aa_ragged_local_f16", (300, 6, 5), 1.0, 0.5, "local", "central", 1.0, "f16", True),
    ("aa_raw_lowmach_bf16", (70, 8, 6), 0.5, 0.25, "lowmach", "raw", 1.0, "bf16", False),
    ("aa_two_wide_f16", (2, 5, 4), 1.0, 0.5, "off", "central", 1.0, "f16", True),
    ("aa_stochastic_bf16sr", (70, 8, 6), 0.5, 0.25, "local", "central", 1.0, "bf16_sr", False),
]


@pytest.mark.parametrize("case", AA_CASES, ids=[c[0] for c in AA_CASES])
def test_aa_pair_step_equals_one_node_step(case):
    """The in-place (AA) 16-bit step with two nodes per thread against its one-node kernel."""
    import paper_2107_14774_amd as P
    name, (nx, ny, nz), r, s, corr, moments, omega_hi, storage, field = case
    _say("case", name)
    p = oracle.Params(nx, ny, nz, r=r, s=s, omega_nu=1.3, omega_xi=1.1, omega_hi=omega_hi, corr=corr,
                      moments=moments)
    f0 = random_state(p, 73)
    g = np.random.Generator(np.random.PCG64(74))
    force = torch.tensor(1e-4 * g.standard_normal((3, *p.shape))).to(torch.float32).cuda() if field else None
    kw = dict(r=p.r, s=p.s, cs2=p.cs2, omega_nu=p.omega_nu, omega_xi=p.omega_xi, omega_hi=p.omega_hi,
              storage=storage, corr=p.corr, moments=p.moments, force=(2e-6, 1e-6, -3e-6), layout="aa")
    with _pairs(False):
        one = P.Lattice(nx, ny, nz, **kw)
    with _pairs(True):
        two = P.Lattice(nx, ny, nz, **kw)
    s1, s2 = one.new_state(), two.new_state()
    one.import_populations(s1, f0.cuda())
    two.import_populations(s2, f0.cuda())
    for n in (2, 6):
        s1, _ = one.step(s1, None, n, force)
        s2, _ = two.step(s2, None, n, force)
        f1, f2 = one.export_populations(s1), two.export_populations(s2)
        _say(f"{name}: max |pairs - one node| = {(f1 - f2).abs().max().item():.3e}")
        assert torch.equal(f1, f2)


FULL_CASES = [
    # name, grid, r, s, moments, storage, force field, mode
    ("full_lagged_f16_field", (256, 6, 5), 1.0, 0.5, "central", "f16", True, "lagged"),
    ("full_exact_bf16", (130, 5, 4), 0.5, 0.25, "central", "bf16", False, "exact"),
    ("full_lagged_raw_bf16sr", (300, 4, 6), 1.0, 0.5, "raw", "bf16_sr", True, "lagged"),
    ("full_lagged_two_wide_f16", (2, 7, 5), 0.75, 1.0, "central", "f16", False, "lagged"),
]


@pytest.mark.parametrize("case", FULL_CASES, ids=[c[0] for c in FULL_CASES])
def test_full_pair_step_equals_one_node_step(case):
    """The full-correction step with two nodes per thread (the pairs' column sums and density output)
    against its one-node kernel, in both time levels of the density gradient: states and density
    fields bit for bit."""
    name, (nx, ny, nz), r, s, moments, storage, field, mode = case
    _say("case", name)
    p = oracle.Params(nx, ny, nz, r=r, s=s, omega_nu=1.4, omega_xi=1.15, corr="full", moments=moments)
    f0 = random_state(p, 75)
    g = np.random.Generator(np.random.PCG64(76))
    force = torch.tensor(1e-4 * g.standard_normal((3, *p.shape))).to(torch.float32).cuda() if field else None
    uniform = (1e-5, -2e-6, 3e-6)
    one = _lattice(p, storage, uniform, pairs=False)
    two = _lattice(p, storage, uniform, pairs=True)
    a1, b1 = one.new_state(), one.new_state()
    a2, b2 = two.new_state(), two.new_state()
    one.import_populations(a1, f0.cuda())
    two.import_populations(a2, f0.cuda())
    d1, e1 = one.density(a1), one.field(1)
    d2, e2 = two.density(a2), two.field(1)
    for n in (1, 4):
        a1, b1, d1, e1 = one.step_full(a1, b1, n, d1, e1, mode, force)
        a2, b2, d2, e2 = two.step_full(a2, b2, n, d2, e2, mode, force)
        f1, f2 = one.export_populations(a1), two.export_populations(a2)
        _say(f"{name}: max |pairs - one node| = {(f1 - f2).abs().max().item():.3e}")
        assert torch.equal(f1, f2)
        if mode == "lagged":
            assert torch.equal(d1, d2)
