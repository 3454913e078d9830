"""Write the FP64-oracle reference of the decaying-flow replica (test infrastructure).

    python tests/golden/make_decaying_replica_fixture.py

The throughput workload's flow (Taylor-Green base plus solenoidal Gaussian
modes 1 <= |k| <= 8 at rms 0.01, Re 1600, r = 1, s = 1/2, local corrections)
on a 64x64x32 replica, run for 1000 steps by the FP64 oracle from
f = f_eq(1, u0).  Stored after 250, 500 and 1000 steps: the totals of mass,
momentum and kinetic energy (sum of rho |u|^2 / 2 over nodes) and the velocity
(eq. 12) at 1024 seeded sample nodes.  Only ``oracle/`` computes these values
(``workloads/`` supplies the seeded initial field); the GPU tests compare their
runs of the same workload against this file.  About 10 minutes on 8 cores.
"""

import json
import os
import sys
import time

import numpy as np
import torch

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
sys.path.insert(0, ROOT)

import oracle  # noqa: E402
from oracle import analytic as A  # noqa: E402
from oracle import lbm as OL  # noqa: E402
import workloads as W  # noqa: E402

OUT = os.path.join(HERE, "decaying_replica_64x64x32.json")
CHECKPOINTS = (250, 500, 1000)
SAMPLES, SAMPLE_SEED = 1024, 61


def main():
    w = W.replica(W.DECAYING_512, 64, 64, 32, steps=CHECKPOINTS[-1])
    p = oracle.Params(w.nx, w.ny, w.nz, r=w.r, s=w.s, cs2=w.cs2, omega_nu=A.omega_from_nu(w.nu, w.cs2),
                      omega_xi=A.omega_from_xi(w.xi, w.cs2), corr="local")
    u0 = torch.from_numpy(W.initial_velocity(w))
    f = OL.init_equilibrium(torch.ones(p.shape, dtype=torch.float64), u0, p)
    nodes = W.sample_indices(SAMPLES, p.n, SAMPLE_SEED)
    rec = {"workload": w.name, "grid": [w.nx, w.ny, w.nz], "r": w.r, "s": w.s, "cs2": w.cs2, "nu": w.nu,
           "xi": w.xi, "corrections": "local", "initial": "f_eq(rho = 1, u0), u0 = workloads.initial_velocity",
           "sample_nodes": [int(i) for i in nodes], "sample_seed": SAMPLE_SEED, "steps": {}}
    t, t0 = 0, time.time()
    for target in CHECKPOINTS:
        f = OL.run(f, p, target - t)
        t = target
        rho, u = OL.observables(f, p)
        un = u.reshape(3, -1)
        rec["steps"][str(t)] = {
            "mass": float(rho.sum()),
            "momentum": [float((rho * u[c]).sum()) for c in range(3)],
            "kinetic_energy": float((0.5 * rho * (u ** 2).sum(0)).sum()),
            "u_sample": [[float(f"{float(un[c, i]):.12e}") for c in range(3)] for i in nodes],
        }
        print(f"step {t}: kinetic energy {rec['steps'][str(t)]['kinetic_energy']:.10e} ({time.time() - t0:.0f} s)",
              flush=True)
    with open(OUT, "w") as fh:
        json.dump(rec, fh)
    print("wrote", OUT)


if __name__ == "__main__":
    main()
