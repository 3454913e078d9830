"""Stability of the central-moment (3DCCM) and raw-moment (3DCRM) schemes on
the cuboid lattice: the lid-driven cubic-cavity tests of arXiv:2107.14774,
Sec. 7, on one MI355X.

mode "umax": for each shear rate omega_nu, the largest lid velocity U that
    keeps the run stable for ``--steps`` steps (100,000 in the paper), on the
    30x40x30 (r = 0.75) and 30x60x30 (r = 0.5) grids with s = 1, cs2 = 0.08
    and every other relaxation rate 1 (the paper's Fig. 8 set-up).
mode "remax": at U = 0.2, cs2 = 0.08, r = 0.5, s = 1, the largest Reynolds
    number U H / nu (smallest viscosity) that stays stable on 40x80x40,
    50x100x50 and 90x180x90 (the Fig. 10 set-up).

A run is stable when its FP64 totals stay finite and max |u| stays below 1
(one lattice length per step) at every check (every ``--check`` steps and at
the end).  Bisection on U (or omega_nu) to ``--iters`` halvings.  The paper
prints these results as figures only, so the comparison is qualitative: the
central scheme should hold larger U (or Re) than the raw one.

    python examples/stability_sweep.py --mode umax
    python examples/stability_sweep.py --mode remax

Prints one JSON object per measured point.
"""

import argparse
import json
import os
import sys
import time

import torch

sys.path.insert(0, os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
import paper_2107_14774_amd as P  # noqa: E402
from paper_2107_14774_amd import _lib  # noqa: E402

CS2 = 0.08


def stable(grid, r, s, omega_nu, U, moments, steps, check, corr="local"):
    nx, ny, nz = grid
    lid = [(0.0, 0.0, 0.0)] * 6
    lid[3] = (U, 0.0, 0.0)
    lat = P.Lattice(nx, ny, nz, r=r, s=s, cs2=CS2, omega_nu=omega_nu, omega_xi=1.0, bc_x="bounceback",
                    bc_y="bounceback", bc_z="bounceback", wall_velocity=lid, moments=moments, corr=corr)
    a, b = lat.new_state(), lat.new_state()
    lat.init(a)
    done = 0
    try:
        while done < steps:
            n = min(check, steps - done)
            a, b = lat.step(a, b, n)
            done += n
            m = lat.moments(a)
            P.lbm_check_sums(m.sums)
            if not (m.u.abs().max().item() < 1.0):
                return False, done
    except _lib.LbmError as e:
        if e.code != _lib.LBM_ENONFINITE:
            raise
        return False, done
    return True, done


def bisect(fn, lo, hi, iters):
    """Largest x in [lo, hi] with fn(x) True, assuming fn(lo) is True; returns (x, runs)."""
    runs = 0
    ok_hi, _ = fn(hi)
    runs += 1
    if ok_hi:
        return hi, runs
    for _ in range(iters):
        mid = 0.5 * (lo + hi)
        ok, _ = fn(mid)
        runs += 1
        lo, hi = (mid, hi) if ok else (lo, mid)
    return lo, runs


def umax_mode(args):
    grids = {"30x40x30": ((30, 40, 30), 0.75, 1.0), "30x60x30": ((30, 60, 30), 0.5, 1.0)}
    omegas = [float(w) for w in args.omegas.split(",")]
    for gname in args.grids.split(","):
        grid, r, s = grids[gname]
        for moments in ("central", "raw"):
            for w in omegas:
                t0 = time.perf_counter()
                u, runs = bisect(lambda U: stable(grid, r, s, w, U, moments, args.steps, args.check),
                                 0.0, args.u_hi, args.iters)
                print(json.dumps({"mode": "umax", "grid": gname, "r": r, "s": s, "cs2": CS2, "scheme": moments,
                                  "omega_nu": w, "U_max": round(u, 5), "resolution": args.u_hi / 2 ** args.iters,
                                  "steps": args.steps, "runs": runs,
                                  "seconds": round(time.perf_counter() - t0, 2)}), flush=True)


def remax_mode(args):
    U = args.U
    for gname in args.grids.split(","):
        nx, ny, nz = (int(v) for v in gname.split("x"))
        r, s = nx / ny, 1.0
        H = nx
        for moments in ("central", "raw"):
            t0 = time.perf_counter()
            w, runs = bisect(lambda om: stable((nx, ny, nz), r, s, om, U, moments, args.steps, args.check),
                             1.0, 1.999, args.iters)
            nu = CS2 * (1.0 / w - 0.5)
            print(json.dumps({"mode": "remax", "grid": gname, "r": r, "s": s, "cs2": CS2, "U": U, "scheme": moments,
                              "omega_nu_max": round(w, 5), "Re_max": round(U * H / nu, 1), "steps": args.steps,
                              "runs": runs, "seconds": round(time.perf_counter() - t0, 2)}), flush=True)


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--mode", choices=("umax", "remax"), default="umax")
    ap.add_argument("--grids", default=None)
    ap.add_argument("--omegas", default="1.0,1.2,1.4,1.6,1.8,1.9")
    ap.add_argument("--steps", type=int, default=100000)
    ap.add_argument("--check", type=int, default=5000)
    ap.add_argument("--iters", type=int, default=7)
    ap.add_argument("--u-hi", type=float, default=0.4)
    ap.add_argument("--U", type=float, default=0.2)
    args = ap.parse_args()
    if not torch.cuda.is_available():
        sys.exit("needs a GPU")
    if args.grids is None:
        args.grids = "30x40x30,30x60x30" if args.mode == "umax" else "40x80x40,50x100x50,90x180x90"
    (umax_mode if args.mode == "umax" else remax_mode)(args)


if __name__ == "__main__":
    main()
