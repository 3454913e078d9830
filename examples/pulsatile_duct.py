"""Pulsatile flow in a square duct (arXiv:2107.14774, Sec. 5.2) on one MI355X.

Duct of side 2a = 40, periodic along x, halfway bounce-back walls in y and
z, driven by F_x = F_m cos(omega t) with F_m = 1e-5 and period T = 10,000
steps, at Womersley numbers Wo = a sqrt(omega/nu) = 3.09 and 6.25, on the
paper's three cuboid grids 40x80x40 (r, s) = (0.5, 1), 40x80x80 (0.5, 0.5)
and 40x160x80 (0.25, 0.5).  cs2 = min(r^2, s^2)/3, bulk viscosity = shear
viscosity.  Each run starts from rest and lasts enough whole periods for
the start-up transient to decay (e^-7 of the slowest duct mode); over the
last period the velocity at eight instants is compared with the periodic
series solution.  The step uses lbm_step_forcing (one uniform force per
step); the force of the current instant is set before reading eq. 12's
velocity.  The series is evaluated here in NumPy (the double eigenfunction
series, summed to 400 x 400 terms).

    python examples/pulsatile_duct.py

Prints one JSON object per case: the largest |u - u_series| over the cross
section and the eight instants, in units of F_m/omega, and the MLUPS of the
stepping alone.
"""

import json
import math
import os
import sys
import time

import numpy as np
import torch

sys.path.insert(0, os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
import paper_2107_14774_amd as P  # noqa: E402

GRIDS = [((40, 80, 40), 0.5, 1.0), ((40, 80, 80), 0.5, 0.5), ((40, 160, 80), 0.25, 0.5)]


def periodic_series(y, z, t, a, F, omega, nu, nterms=400):
    """u_x of the periodic state: sum over odd m, n of
    (F) 16 (-1)^((m-1)/2+(n-1)/2) / (pi^2 m n) cos(m pi y/2a) cos(n pi z/2a) / (i omega + nu lambda_mn)."""
    odd = np.arange(1, 2 * nterms, 2, dtype=np.float64)
    k = odd * math.pi / (2.0 * a)
    sign = np.where(((odd - 1) // 2) % 2 == 1, -1.0, 1.0)
    cy = np.cos(np.multiply.outer(y, k)) * (sign / odd)
    cz = np.cos(np.multiply.outer(z, k)) * (sign / odd)
    coef = (16.0 / math.pi ** 2) * F / (1j * omega + nu * (k[:, None] ** 2 + k[None, :] ** 2))
    return np.real(np.einsum("...m,mn,...n->...", cy, coef, cz) * np.exp(1j * omega * t))


def run(grid, r, s, Wo, a=20.0, F=1e-5, T=10000):
    nx, ny, nz = grid
    omega = 2 * math.pi / T
    nu = a * a * omega / Wo ** 2
    cs2 = min(r * r, s * s) / 3.0
    on, ox = P.relaxation_rates(nu, nu, cs2)
    lat = P.Lattice(nx, ny, nz, r=r, s=s, cs2=cs2, omega_nu=on, omega_xi=ox, bc_y="bounceback", bc_z="bounceback")
    a_state, b_state = lat.new_state(), lat.new_state()
    lat.init(a_state)
    slowest = nu * 2.0 * (math.pi / (2.0 * a)) ** 2
    periods = int(math.ceil(7.0 / (slowest * T))) + 1
    Y, Z = np.meshgrid((np.arange(ny) + 0.5) * r - a, (np.arange(nz) + 0.5) * s - a)
    t_series = np.arange(periods * T, dtype=np.float64)
    forces = np.zeros((periods * T, 3))
    forces[:, 0] = F * np.cos(omega * t_series)
    # everything but the last period in one call, then the last period in eighths;
    # only the stepping is timed (the series is evaluated on the host in between)
    wall = 0.0

    def advance(a_state, b_state, chunk):
        nonlocal wall
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        a_state, b_state = lat.step_forcing(a_state, b_state, chunk)
        torch.cuda.synchronize()
        wall += time.perf_counter() - t0
        return a_state, b_state

    n0 = (periods - 1) * T
    a_state, b_state = advance(a_state, b_state, forces[:n0])
    worst, n = 0.0, n0
    for k in range(8):
        n1 = n0 + (k + 1) * T // 8
        a_state, b_state = advance(a_state, b_state, forces[n:n1])
        n = n1
        lat.set_force((F * math.cos(omega * n), 0.0, 0.0))
        u = lat.moments(a_state, sums=False).u[0].double().cpu().numpy()   # (nz, ny, nx)
        want = periodic_series(Y, Z, n, a, F, omega, nu)
        worst = max(worst, float(np.abs(u - want[:, :, None]).max() / (F / omega)))
    return {"grid": list(grid), "r": r, "s": s, "Wo": Wo, "nu": nu, "cs2": cs2, "periods": periods, "steps": n,
            "max_err_over_F_omega": worst, "mlups": lat.n * n / wall / 1e6}


def main():
    if not torch.cuda.is_available():
        sys.exit("needs a GPU")
    for Wo in (3.09, 6.25):
        for grid, r, s in GRIDS:
            print(json.dumps(run(grid, r, s, Wo)), flush=True)


if __name__ == "__main__":
    main()
