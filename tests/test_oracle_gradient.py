"""Pins of the gradient oracle: dot-product tests against finite-difference
directional derivatives and central finite differences of a multi-step loss."""

import numpy as np
import pytest
import torch

import oracle
from oracle import gradient as G
from oracle import lbm
import workloads as W

DT = torch.float64


def _state(p, seed, amp=0.03):
    g = np.random.Generator(np.random.PCG64(seed))
    u = torch.tensor(amp * g.standard_normal((3, *p.shape)))
    rho = torch.tensor(1.0 + 0.01 * g.standard_normal(p.shape))
    f = lbm.init_equilibrium(rho, u, p)
    f = f * (1.0 + torch.tensor(1e-3 * g.standard_normal(f.shape)))
    force = torch.tensor(1e-4 * g.standard_normal((3, *p.shape)))
    return f, force, g


@pytest.mark.parametrize("bc", ["periodic", "bounceback"])
@pytest.mark.parametrize("corr", ["local", "lowmach"])
def test_step_vjp_dot_product(bc, corr):
    p = oracle.Params(5, 4, 6, r=0.5, s=0.25, omega_nu=1.5, omega_xi=1.2, corr=corr, bc_y=bc, bc_z=bc)
    f, force, g = _state(p, 3)
    v = torch.tensor(g.standard_normal(f.shape)) * 1e-3
    vF = torch.tensor(g.standard_normal(force.shape)) * 1e-5
    w = torch.tensor(g.standard_normal(f.shape))
    h = 1e-3
    jv = (lbm.step(f + h * v, p, force + h * vF) - lbm.step(f - h * v, p, force - h * vF)) / (2 * h)
    lam_f, lam_F = G.step_vjp(f, p, force, w)
    lhs = (jv * w).sum()
    rhs = (v * lam_f).sum() + (vF * lam_F).sum()
    assert abs(lhs - rhs) <= 1e-9 * abs(lhs), (lhs.item(), rhs.item())


def test_observables_and_init_vjp():
    p = oracle.Params(3, 4, 2, r=0.8, s=0.5)
    f, force, g = _state(p, 4)
    gr = torch.tensor(g.standard_normal(p.shape))
    gu = torch.tensor(g.standard_normal((3, *p.shape)))
    v = torch.tensor(g.standard_normal(f.shape)) * 1e-3
    h = 1e-3
    r1, u1 = lbm.observables(f + h * v, p, force)
    r2, u2 = lbm.observables(f - h * v, p, force)
    lhs = (((r1 - r2) * gr).sum() + ((u1 - u2) * gu).sum()) / (2 * h)
    rhs = (G.observables_vjp(f, p, force, gr, gu) * v).sum()
    assert abs(lhs - rhs) <= 1e-9 * abs(lhs)
    rho = torch.tensor(1 + 0.01 * g.standard_normal(p.shape))
    u = torch.tensor(0.03 * g.standard_normal((3, *p.shape)))
    lam = torch.tensor(g.standard_normal(f.shape))
    dr = torch.tensor(g.standard_normal(p.shape)) * 1e-3
    du = torch.tensor(g.standard_normal((3, *p.shape))) * 1e-3
    lhs = ((lbm.init_equilibrium(rho + h * dr, u + h * du, p)
            - lbm.init_equilibrium(rho - h * dr, u - h * du, p)) * lam).sum() / (2 * h)
    g_rho, g_u = G.init_vjp(rho, u, p, lam)
    rhs = (g_rho * dr).sum() + (g_u * du).sum()
    assert abs(lhs - rhs) <= 1e-9 * abs(lhs)


def test_loss_gradient_matches_central_differences():
    """dL/dF and dL/du0 of a 12-step duct run vs central differences on sampled entries."""
    w = W.replica(W.ADJOINT_DUCT_128, 6, 8, 6, steps=12)
    p = oracle.Params(w.nx, w.ny, w.nz, r=w.r, s=w.s, cs2=w.cs2,
                      omega_nu=oracle.analytic.omega_from_nu(w.nu, w.cs2),
                      omega_xi=oracle.analytic.omega_from_xi(w.xi, w.cs2),
                      bc_y=w.bc_y, bc_z=w.bc_z)
    g = np.random.Generator(np.random.PCG64(7))
    force = torch.tensor(1e-5 * g.standard_normal((3, *p.shape)))
    u0 = torch.tensor(1e-3 * g.standard_normal((3, *p.shape)))
    rho0 = torch.ones(p.shape, dtype=DT)
    target = torch.tensor(1e-3 * g.standard_normal((3, *p.shape)))
    L, gF, gu = G.loss_and_gradients(p, rho0, u0, force, target, w.steps)
    idx = W.sample_indices(6, force.numel(), 41)
    for flat in idx:
        c = np.unravel_index(flat, force.shape)
        h = 1e-6
        Fp, Fm = force.clone(), force.clone()
        Fp[c] += h
        Fm[c] -= h
        fd = (G.loss(p, rho0, u0, Fp, target, w.steps) - G.loss(p, rho0, u0, Fm, target, w.steps)) / (2 * h)
        assert abs(fd - gF[c]) <= 1e-6 * abs(gF).max(), (c, fd.item(), gF[c].item())
        up, um = u0.clone(), u0.clone()
        up[c] += h
        um[c] -= h
        fd = (G.loss(p, rho0, up, force, target, w.steps) - G.loss(p, rho0, um, force, target, w.steps)) / (2 * h)
        assert abs(fd - gu[c]) <= 1e-6 * abs(gu).max(), (c, fd.item(), gu[c].item())
