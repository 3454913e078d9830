"""Write the FP64-oracle reference of a long-trajectory gradient (test infrastructure).

    python tests/golden/make_c5_gradient_fixture.py

The FP16 adjoint workload's physics (r = 1/2, s = 1/4, cs2 = 1/48, tau_nu =
tau_xi = 0.8, periodic) on a 32x32x16 replica: u0 = solenoidal modes
1 <= |n| <= 3 at rms 0.02 (seed 5), target u* the same with seed 50,
L = 1/2 sum over nodes of |u(T) - u*|^2 after T = 1000 steps (the workload's
step count).  The oracle runs forward keeping every state, then takes its
one-step vector-Jacobian products in reverse (the chain rule over
oracle.gradient's observables_vjp, step_vjp and init_vjp).  Stored: L, the L2
norm of dL/du0, and dL/du0 at 1024 seeded nodes.  Only ``oracle/`` computes
these values (``workloads/`` supplies the seeded fields).  About 10 minutes on
8 cores and 4 GB of memory.
"""

import json
import os
import sys
import time

import torch

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
sys.path.insert(0, ROOT)

import oracle  # noqa: E402
from oracle import analytic as A  # noqa: E402
from oracle import gradient as G  # noqa: E402
from oracle import lbm as OL  # noqa: E402
import workloads as W  # noqa: E402

OUT = os.path.join(HERE, "c5_gradient_replica_32x32x16.json")
GRID, STEPS, KMAX = (32, 32, 16), 1000, 3
SAMPLES, SAMPLE_SEED = 1024, 71
DT = torch.float64


def main():
    w = W.ADJOINT_F16_384
    nx, ny, nz = GRID
    p = oracle.Params(nx, ny, nz, r=w.r, s=w.s, cs2=w.cs2, omega_nu=A.omega_from_nu(w.nu, w.cs2),
                      omega_xi=A.omega_from_xi(w.xi, w.cs2), corr="local")
    u0 = torch.from_numpy(W.random_modes(nx, ny, nz, p.r, p.s, KMAX, w.extra["rms"], w.extra["seed"]))
    target = torch.from_numpy(W.random_modes(nx, ny, nz, p.r, p.s, KMAX, w.extra["target_rms"],
                                             w.extra["target_seed"]))
    rho0 = torch.ones(p.shape, dtype=DT)
    force = torch.zeros(3, *p.shape, dtype=DT)
    t0 = time.time()
    states = [OL.init_equilibrium(rho0, u0, p)]
    for t in range(STEPS):
        states.append(OL.step(states[-1], p, force=force))
        if (t + 1) % 250 == 0:
            print(f"forward {t + 1} ({time.time() - t0:.0f} s)", flush=True)
    _, u_T = OL.observables(states[-1], p, force=force)
    loss = float(0.5 * ((u_T - target) ** 2).sum())
    lam = G.observables_vjp(states[-1], p, force, torch.zeros(p.shape, dtype=DT), u_T - target)
    for t in range(STEPS - 1, -1, -1):
        lam, _ = G.step_vjp(states[t], p, force, lam)
        states[t + 1] = None
        if t % 250 == 0:
            print(f"reverse at step {t} ({time.time() - t0:.0f} s)", flush=True)
    _, g_u0 = G.init_vjp(rho0, u0, p, lam)
    nodes = W.sample_indices(SAMPLES, p.n, SAMPLE_SEED)
    gu = g_u0.reshape(3, -1)
    rec = {"workload": "adjoint_f16_384x384x192 physics on a 32x32x16 replica", "grid": list(GRID), "r": p.r,
           "s": p.s, "cs2": p.cs2, "nu": w.nu, "xi": w.xi, "steps": STEPS, "kmax": KMAX,
           "u0": {"rms": w.extra["rms"], "seed": w.extra["seed"]},
           "target": {"rms": w.extra["target_rms"], "seed": w.extra["target_seed"]},
           "loss": loss, "grad_u0_l2": float(g_u0.norm()), "sample_seed": SAMPLE_SEED,
           "sample_nodes": [int(i) for i in nodes],
           "grad_u0_sample": [[float(f"{float(gu[c, i]):.12e}") for c in range(3)] for i in nodes]}
    with open(OUT, "w") as fh:
        json.dump(rec, fh)
    print(f"L = {loss:.6e}, |dL/du0| = {rec['grad_u0_l2']:.6e} ({time.time() - t0:.0f} s)")
    print("wrote", OUT)


if __name__ == "__main__":
    main()
