"""Lid-driven shallow cavity: cubic versus cuboid lattice (the computational-
advantage study of arXiv:2107.14774, Sec. 6), on one MI355X.

Cavity L x H x W with L/H = 4, W/H = 2; the lid y = H moves along x at U;
Re = U L / nu = 100.  Ny = 64 nodes across the height in every case:

    cubic   256 x 64 x 128   r = 1,     s = 1     cs2 = 1/3
    (i)     104 x 64 x 40    r = 0.406, s = 1.3   cs2 = 0.04
    (ii)     96 x 64 x 64    r = 0.375, s = 0.75  cs2 = 0.04
    (iii)    96 x 64 x 48    r = 0.375, s = 1.0   cs2 = 0.04

(r, s as printed; the grids follow from Nx = r (L/H) Ny, Nz = (r/s)(W/H) Ny,
so case (i) uses r = 26/64 exactly.)  Every case runs from rest to a steady
state (largest change of u over ``--check-every`` steps below ``--tol`` U)
with FP32 storage and the local corrections, then reports nodes, state
memory, steps, wall time, MLUPS and the centreline profiles u(y) at
x = L/2, z = W/2 and v(x) at y = H/2, z = W/2 against the cubic run.

    python examples/shallow_cavity.py [--cases cubic,i,ii,iii] [--tol 1e-6]

Prints one JSON object per case, then one summary object.
"""

import argparse
import json
import os
import sys
import time

import numpy as np
import torch

sys.path.insert(0, os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
import paper_2107_14774_amd as P  # noqa: E402

RE = 100.0
CASES = {
    "cubic": dict(nx=256, ny=64, nz=128, r=1.0, s=1.0, cs2=1.0 / 3.0, U=0.1),
    "i": dict(nx=104, ny=64, nz=40, r=26.0 / 64.0, s=1.3, cs2=0.04, U=0.035),
    "ii": dict(nx=96, ny=64, nz=64, r=0.375, s=0.75, cs2=0.04, U=0.035),
    "iii": dict(nx=96, ny=64, nz=48, r=0.375, s=1.0, cs2=0.04, U=0.035),
}


def centre_pair(n):
    """Indices whose mean is the mid-plane value (cell centres at (i + 1/2)/n)."""
    return (n // 2 - 1, n // 2) if n % 2 == 0 else (n // 2, n // 2)


def run_case(name, tol, check_every, max_steps):
    c = CASES[name]
    nu = c["U"] * c["nx"] / RE                       # L = nx in x-lengths
    on, ox = P.relaxation_rates(nu, nu, c["cs2"])
    lid = [(0.0, 0.0, 0.0)] * 6
    lid[3] = (c["U"], 0.0, 0.0)
    lat = P.Lattice(c["nx"], c["ny"], c["nz"], r=c["r"], s=c["s"], cs2=c["cs2"], omega_nu=on, omega_xi=ox,
                    bc_x="bounceback", bc_y="bounceback", bc_z="bounceback", wall_velocity=lid)
    a, b = lat.new_state(), lat.new_state()
    lat.init(a)
    u_prev = lat.moments(a, sums=False).u.clone()
    steps, change = 0, float("inf")
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    while steps < max_steps:
        a, b = lat.step(a, b, check_every)
        steps += check_every
        u = lat.moments(a, sums=False).u
        change = (u - u_prev).abs().max().item() / c["U"]
        u_prev.copy_(u)
        if change < tol:
            break
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    m = lat.moments(a)
    sums = P.lbm_check_sums(m.sums)
    u = m.u.double().cpu().numpy() / c["U"]          # (3, nz, ny, nx)
    zc, yc, xc = centre_pair(c["nz"]), centre_pair(c["ny"]), centre_pair(c["nx"])
    u_of_y = 0.25 * sum(u[0, z, :, x] for z in zc for x in xc)
    v_of_x = 0.25 * sum(u[1, z, y, :] for z in zc for y in yc)
    return {
        "case": name, "grid": [c["nx"], c["ny"], c["nz"]], "r": c["r"], "s": c["s"], "cs2": c["cs2"],
        "U": c["U"], "nu": nu, "nodes": lat.n, "state_bytes_two_buffers": 2 * lat.h.state_bytes,
        "steps": steps, "converged": change < tol, "last_change": change, "wall_s": wall,
        "mlups": lat.n * steps / wall / 1e6, "mass": sums[0],
        "y": ((np.arange(c["ny"]) + 0.5) / c["ny"]).tolist(), "u_of_y": u_of_y.tolist(),
        "x": ((np.arange(c["nx"]) + 0.5) / c["nx"]).tolist(), "v_of_x": v_of_x.tolist(),
    }


def compare(ref, res):
    """Largest profile differences (in units of U) against the reference run."""
    du = np.max(np.abs(np.interp(ref["y"], res["y"], res["u_of_y"]) - np.asarray(ref["u_of_y"])))
    dv = np.max(np.abs(np.interp(res["x"], ref["x"], ref["v_of_x"]) - np.asarray(res["v_of_x"])))
    return float(du), float(dv)


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--cases", default="cubic,i,ii,iii")
    ap.add_argument("--tol", type=float, default=1e-6)
    ap.add_argument("--check-every", type=int, default=1000)
    ap.add_argument("--max-steps", type=int, default=400000)
    args = ap.parse_args()
    if not torch.cuda.is_available():
        sys.exit("needs a GPU")
    results = {}
    for name in [c for c in args.cases.split(",") if c]:
        res = run_case(name, args.tol, args.check_every, args.max_steps)
        results[name] = res
        brief = {k: v for k, v in res.items() if k not in ("y", "u_of_y", "x", "v_of_x")}
        print(json.dumps(brief), flush=True)
    summary = {}
    if "cubic" in results:
        ref = results["cubic"]
        for name, res in results.items():
            if name == "cubic":
                continue
            du, dv = compare(ref, res)
            summary[name] = {"node_ratio": ref["nodes"] / res["nodes"],
                             "time_ratio": ref["wall_s"] / res["wall_s"],
                             "max_du_over_U": du, "max_dv_over_U": dv}
    print(json.dumps({"summary_vs_cubic": summary}), flush=True)


if __name__ == "__main__":
    main()
