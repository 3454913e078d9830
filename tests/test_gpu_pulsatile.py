"""GPU parity of time-dependent forcing (the pulsatile duct of Sec. 5.2): lbm_step_forcing
and lbm_set_force against the FP64 oracle, and the full-size duct against the periodic series."""

import math
import sys

import numpy as np
import pytest
import torch

import oracle
from oracle import analytic as A
from oracle import lbm as OL
from helpers import gpu_lattice, rel_l2

pytestmark = pytest.mark.gpu
DT = torch.float64


def _say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def _duct(a, r, s, Wo, nu, nx=2):
    ny, nz = int(round(2 * a / r)), int(round(2 * a / s))
    cs2 = min(r * r, s * s) / 3
    om = A.omega_from_nu(nu, cs2)
    p = oracle.Params(nx, ny, nz, r=r, s=s, cs2=cs2, omega_nu=om, omega_xi=om, bc_y="bounceback", bc_z="bounceback")
    return p, (Wo / a) ** 2 * nu


def test_time_dependent_force_matches_oracle():
    """300 steps of a pulsatile duct replica (2 x 16 x 8, r = 1/2, s = 1) with one force per step."""
    F = 1e-5
    p, w = _duct(4.0, 0.5, 1.0, 3.09, 0.04)
    forces = np.zeros((300, 3))
    forces[:, 0] = F * np.cos(w * np.arange(300))
    lat = gpu_lattice(p)
    a, b = lat.new_state(), lat.new_state()
    lat.init(a)
    cur, _ = lat.step_forcing(a, b, forces)
    lat.set_force((F * math.cos(w * 300), 0.0, 0.0))
    u = lat.moments(cur).u.cpu()
    f = OL.init_equilibrium(torch.ones(p.shape, dtype=DT), torch.zeros(3, *p.shape, dtype=DT), p)
    for n in range(300):
        f = OL.step(f, p, force=tuple(forces[n]))
    _, uo = OL.observables(f, p, force=(F * math.cos(w * 300), 0.0, 0.0))
    err = rel_l2(u, uo)
    # the same run stepped one call at a time through lbm_set_force is bit-identical
    a2, b2 = lat.new_state(), lat.new_state()
    lat.init(a2)
    for n in range(300):
        lat.set_force(tuple(forces[n]))
        a2, b2 = lat.step(a2, b2, 1)
    same = torch.equal(lat.export_populations(a2), lat.export_populations(cur))
    _say(f"pulsatile replica 300 steps: rel L2(u) = {err:.3e}; set_force loop bit-identical: {same}")
    assert err <= 1e-5
    assert same


def test_full_size_pulsatile_duct_follows_the_series():
    """The 40x80x40 duct of Sec. 5.2 (2a = 40, r = 1/2, s = 1, Wo = 3.09, T = 10,000 steps),
    three periods from rest; over the last one u stays within 1% of F_m/omega of the series."""
    F, T, a = 1e-5, 10000, 20.0
    w = 2 * math.pi / T
    nu = a * a * w / 3.09 ** 2
    p, _ = _duct(a, 0.5, 1.0, 3.09, nu, nx=40)
    lat = gpu_lattice(p)
    st, sc = lat.new_state(), lat.new_state()
    lat.init(st)
    n_all = 3 * T
    forces = np.zeros((n_all, 3))
    forces[:, 0] = F * np.cos(w * np.arange(n_all))
    st, sc = lat.step_forcing(st, sc, forces[:2 * T])
    Y, Z = np.meshgrid((np.arange(p.ny) + 0.5) * p.r - a, (np.arange(p.nz) + 0.5) * p.s - a)
    worst, n = 0.0, 2 * T
    for k in range(4):
        n1 = 2 * T + (k + 1) * T // 4
        st, sc = lat.step_forcing(st, sc, forces[n:n1])
        n = n1
        lat.set_force((F * math.cos(w * n), 0.0, 0.0))
        u = lat.moments(st, sums=False).u[0].double().cpu().numpy()
        want = A.pulsatile_duct_double_series(Y, Z, n, a, a, F, w, 1.0, nu)
        worst = max(worst, float(np.abs(u - want[:, :, None]).max() / (F / w)))
    _say(f"full-size pulsatile duct: max |u - series| / (F/omega) = {worst:.3e}")
    assert worst < 0.01
