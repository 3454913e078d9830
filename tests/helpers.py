"""Shared helpers of the test suite (test infrastructure; imports the oracle)."""

import numpy as np
import torch

import oracle
from oracle import analytic as A
from oracle import equilibrium as EQ
from oracle import lbm as OL

DT = torch.float64


def oracle_params(w, corr="local", nx=None, ny=None, nz=None):
    return oracle.Params(nx or w.nx, ny or w.ny, nz or w.nz, r=w.r, s=w.s, cs2=w.cs2,
                         omega_nu=A.omega_from_nu(w.nu, w.cs2), omega_xi=A.omega_from_xi(w.xi, w.cs2),
                         corr=corr, bc_y=w.bc_y, bc_z=w.bc_z)


def gpu_lattice(p, storage="f32", force=(0.0, 0.0, 0.0), rho0=1.0):
    """HIP lattice with the same parameters as the oracle Params ``p``."""
    import paper_2107_14774_amd as P
    return P.Lattice(p.nx, p.ny, p.nz, r=p.r, s=p.s, cs2=p.cs2, omega_nu=p.omega_nu, omega_xi=p.omega_xi,
                     omega_hi=p.omega_hi,
                     bc_x=p.bc_x, bc_y=p.bc_y, bc_z=p.bc_z, storage=storage, corr=p.corr, rho0=rho0,
                     force=force, wall_velocity=p.wall_velocity, moments=p.moments)


def fp32_rounded_state(f, p, rho0=1.0):
    """f with its deviations from w rho0 rounded to float32 (the FP32 storage format)."""
    w = EQ.rest_weights(p.r, p.s, p.cs2)[:, None, None, None] * rho0
    dev = (f - w).to(torch.float32).to(DT)
    return w + dev


def random_state(p, seed, mach=0.1, rho_amp=0.02, noise=1e-3):
    """f_eq of random rho, u (u ~ N(0, (mach cs)^2) per component) with relative noise."""
    g = np.random.Generator(np.random.PCG64(seed))
    u_amp = mach * float(np.sqrt(p.cs2))
    rho = torch.tensor(1.0 + rho_amp * g.standard_normal(p.shape))
    u = torch.tensor(u_amp * g.standard_normal((3, *p.shape)))
    f = OL.init_equilibrium(rho, u, p)
    f = f * (1.0 + torch.tensor(noise * g.standard_normal(f.shape)))
    return f


def rel_l2(a, b):
    a = torch.as_tensor(a, dtype=DT).cpu()
    b = torch.as_tensor(b, dtype=DT).cpu()
    return float((a - b).norm() / b.norm())
