"""Reverse mode through the oracle (test infrastructure only).

The step of ``oracle.lbm`` is written in plain differentiable torch ops, so
torch's autograd gives its exact FP64 vector-Jacobian products.  This module
packages the ones the adjoint path needs:

* ``step_vjp``          -- (d step / d f)^T lam and (d step / d F)^T lam for one step
* ``observables_vjp``   -- (d (rho, u) / d f)^T (g_rho, g_u) (eq. 12)
* ``init_vjp``          -- (d f_eq / d (rho, u))^T lam
* ``loss_and_gradients``-- L = 1/2 sum |u(T) - u*|^2 after T steps from
                           f_eq(rho0, u0) under a per-node force, with
                           dL/dF (per node) and dL/du0.
The finite-difference checks of these live in the tests.
"""

import torch

from . import lbm
from .params import Params

DT = torch.float64


def step_vjp(f, p: Params, force_field, lam):
    """(lam_f, lam_F) = VJP of one step at (f, force_field) with cotangent lam.

    ``f`` (27, nz, ny, nx), ``force_field`` (3, nz, ny, nx), ``lam`` like f.
    """
    f = f.detach().clone().requires_grad_(True)
    F = force_field.detach().clone().requires_grad_(True)
    out = lbm.step(f, p, force=F)
    gf, gF = torch.autograd.grad(out, (f, F), grad_outputs=lam)
    return gf, gF


def observables_vjp(f, p: Params, force_field, g_rho, g_u):
    f = f.detach().clone().requires_grad_(True)
    rho, u = lbm.observables(f, p, force=force_field)
    (gf,) = torch.autograd.grad((rho, u), (f,), grad_outputs=(g_rho, g_u))
    return gf


def init_vjp(rho, u, p: Params, lam):
    rho = rho.detach().clone().requires_grad_(True)
    u = u.detach().clone().requires_grad_(True)
    f = lbm.init_equilibrium(rho, u, p)
    g_rho, g_u = torch.autograd.grad(f, (rho, u), grad_outputs=lam)
    return g_rho, g_u


def loss(p: Params, rho0, u0, force_field, target, nsteps, lagged=False):
    """L = 1/2 sum over nodes and components of (u(T) - u*)^2.  ``lagged``: the
    full corrections' density gradient one step behind (``lbm.run``)."""
    f = lbm.run(lbm.init_equilibrium(rho0, u0, p), p, nsteps, force_field, lagged=lagged)
    _, u = lbm.observables(f, p, force=force_field)
    return 0.5 * ((u - target) ** 2).sum()


def loss_and_gradients(p: Params, rho0, u0, force_field, target, nsteps, lagged=False):
    """(L, dL/dforce_field, dL/du0) through the whole trajectory, FP64."""
    u0 = torch.as_tensor(u0, dtype=DT).detach().clone().requires_grad_(True)
    F = torch.as_tensor(force_field, dtype=DT).detach().clone().requires_grad_(True)
    L = loss(p, torch.as_tensor(rho0, dtype=DT), u0, F, torch.as_tensor(target, dtype=DT), nsteps, lagged)
    gF, gu = torch.autograd.grad(L, (F, u0))
    return L.detach(), gF, gu
