"""Pins of the oracle's wall treatment (Sec. 4): halfway bounce-back on every
axis and the momentum-augmented bounce-back of moving walls.

* plane Couette flow between a stationary and a moving face is an exact steady
  solution of the Navier-Stokes equations with a linear profile; with the
  walls half a cell outside the first and last node the scheme keeps it to
  rounding, for every face normal and wall direction, on a cuboid grid and at
  a density different from rho0 (the wall equilibrium takes the fluid density);
* a planted mistake in the wall equilibrium (r and s exchanged) breaks it;
* one step of a fluid at rest next to a lid moving along x reproduces the
  coefficients printed in eq. 69 (with f_25 paired with f~_20, the erratum of
  that equation);
* a closed lid-driven cavity keeps its mass (the wall terms cancel in pairs,
  also at the edges where the lid meets the side walls).
"""

import math

import pytest
import torch

import oracle
from oracle import equilibrium as EQ
from oracle import lattice as L
from oracle import lbm as OL
from oracle import streaming as ST

DT = torch.float64
AX = "xyz"


def couette_params(normal, tang, U, r=1.0, s=0.5, n_normal=12, omega=1.1):
    n = [2, 2, 2]
    n[AX.index(normal)] = n_normal
    bc = {a: ("bounceback" if a == normal else "periodic") for a in AX}
    wv = [[0.0] * 3 for _ in range(6)]
    wv[2 * AX.index(normal) + 1][AX.index(tang)] = U
    return oracle.Params(n[0], n[1], n[2], r=r, s=s, omega_nu=omega, omega_xi=omega, corr="local",
                         bc_x=bc["x"], bc_y=bc["y"], bc_z=bc["z"], wall_velocity=tuple(map(tuple, wv)))


def couette_error(normal, tang, U=0.02, rho=1.1, steps=400, **kw):
    """max |u - u_exact| / U after ``steps`` steps started from the exact linear profile."""
    p = couette_params(normal, tang, U, **kw)
    N = (p.nx, p.ny, p.nz)[AX.index(normal)]
    prof = U * (torch.arange(N, dtype=DT) + 0.5) / N
    shape = [1, 1, 1]
    shape[2 - AX.index(normal)] = N
    u = torch.zeros(3, *p.shape, dtype=DT)
    u[AX.index(tang)] = prof.reshape(shape).expand(p.shape)
    f = OL.init_equilibrium(torch.full(p.shape, rho, dtype=DT), u, p)
    f = OL.run(f, p, steps)
    _, uu = OL.observables(f, p)
    want = torch.zeros_like(uu)
    want[AX.index(tang)] = u[AX.index(tang)]
    return (uu - want).abs().max().item() / U


@pytest.mark.parametrize("normal,tang", [("y", "x"), ("y", "z"), ("z", "x"), ("x", "y"), ("x", "z")])
def test_couette_flow_is_kept_exactly(normal, tang):
    assert couette_error(normal, tang) < 1e-11


def test_couette_with_a_planted_wall_mistake_fails(monkeypatch):
    real = EQ.feq
    monkeypatch.setattr(ST.EQ, "feq", lambda rho, u, r, s, cs2: real(rho, u, s, r, cs2))
    assert couette_error("y", "x", r=0.5, s=1.0, steps=200) > 1e-3


def test_one_step_at_rest_gives_the_coefficients_of_eq_69():
    r, s, U, rho = 0.5, 0.8, 0.03, 1.07
    cs2 = 0.1
    wv = ((0, 0, 0), (0, 0, 0), (0, 0, 0), (U, 0, 0), (0, 0, 0), (0, 0, 0))
    p = oracle.Params(3, 4, 3, r=r, s=s, cs2=cs2, omega_nu=1.3, omega_xi=1.2, bc_y="bounceback",
                      wall_velocity=wv)
    f = OL.init_equilibrium(torch.full(p.shape, rho, dtype=DT), torch.zeros(3, *p.shape, dtype=DT), p)
    g = OL.step(f, p)
    top = g[:, :, -1, :]                      # the node row next to the lid
    w = EQ.rest_weights(r, s, cs2) * rho
    k1 = (cs2 - s * s) * cs2 / (2 * r * r * s * s) * rho * U
    k2 = cs2 * cs2 / (4 * r * r * s * s) * rho * U
    # eq. 69: incoming = outgoing value at rest (w rho) plus the printed momentum term
    printed = {4: 0.0, 16: 0.0, 18: 0.0, 9: -k1, 10: k1, 21: k2, 22: -k2, 25: k2, 26: -k2}
    for a, extra in printed.items():
        assert L.EY[a] == -1
        assert torch.allclose(top[a], torch.full_like(top[a], float(w[a] + extra)), rtol=0, atol=2e-15), a
    # every other population at the lid row is the plain rest value
    for a in range(27):
        if a not in printed:
            assert torch.allclose(top[a], torch.full_like(top[a], float(w[a])), rtol=0, atol=2e-15), a


def test_lid_driven_cavity_keeps_its_mass():
    U = 0.05
    p = oracle.Params(10, 8, 6, r=0.5, s=1.0, omega_nu=1.5, omega_xi=1.3, corr="local",
                      bc_x="bounceback", bc_y="bounceback", bc_z="bounceback",
                      wall_velocity=((0, 0, 0),) * 3 + ((U, 0, 0.3 * U),) + ((0, 0, 0),) * 2)
    f = OL.init_equilibrium(torch.ones(p.shape, dtype=DT), torch.zeros(3, *p.shape, dtype=DT), p)
    m0 = f.sum().item()
    f = OL.run(f, p, 150)
    rho, u = OL.observables(f, p)
    assert abs(f.sum().item() - m0) / m0 < 1e-13
    assert u[0].abs().max().item() > 0.1 * U          # the lid drives a flow
