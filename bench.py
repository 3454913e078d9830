"""Benchmark of the fused cuboid D3Q27 collide-and-stream step on one MI355X.

    python bench.py [--gpus 1] [--steps K] [--warmup W] [--variants f32,f16,...] [--no-cpu-baseline]

Variants: f32, f16, bf16, bf16_sr (the step per storage format), full_f32,
full_f16 (full corrections, lagged gradient), aa_f32, aa_f16 (in-place AA
layout), adjoint_f32, adjoint_f32_hbm, adjoint_f16 (the adjoint workloads),
adjoint_full_f32, adjoint_full_lagged_f32 (the adjoint of the full corrections on the
512x512x128 duct, exact and lagged time levels).

Workload: the decaying Taylor-Green + random-mode flow on the periodic
512x512x256 cuboid grid (r = 1, s = 1/2, Re 1600), inputs resident in HBM
before the timed region.  One "step" is one lbm_step launch (gather and
stream, raw moments, scaling, central moments, collision with the cuboid
corrections, inverse maps, store) over every node.  `value` is the FP32
throughput in MLUPS (million lattice-node updates per second); the 16-bit
deviation-storage variants and the adjoint step are reported beside it.

The roofline object prices the dominant kernel (the FP32 step) against the
8 TB/s HBM peak with its algorithmic traffic of 216 bytes per node update
(27 populations read and written once, 4 bytes each); its launch time comes
from HIP events recorded on the stream the kernel runs on.  `traffic` is the
measured HBM traffic per launch from the committed rocprofv3 counter summary,
or null when the kernel sources changed since it was taken.  Two measured
ceilings sit beside the peak: the library's plain copy (lbm_copy, 16 bytes per
thread) and streaming only (lbm_stream: the step's gather and store without
the collision, the same bytes in the same pattern and launch shape).

The CPU baseline times the FP64 oracle (test infrastructure, untuned) on a
bounded replica of the same workload on the host's cores.
"""

import argparse
import hashlib
import json
import math
import os
import re
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

import numpy as np  # noqa: E402
import torch  # noqa: E402

import workloads as W  # noqa: E402

HBM_PEAK_GBS = 8000.0
BYTES_PER_LUP = {"f32": 216, "f16": 108, "bf16": 108, "bf16_sr": 108,
                 # full corrections, lagged density gradient: + write and read of the density deviation field
                 "full_f32": 216 + 8, "full_f16": 108 + 8,
                 # exact density gradient: + a density pass (one more state read, one field write)
                 "full_f32_exact": 216 + 4 + 108 + 4}
FULL_VARIANTS = {"full_f32": ("f32", "lagged"), "full_f16": ("f16", "lagged"), "full_f32_exact": ("f32", "exact")}
# in-place AA layout (one buffer): same bytes per update, half the memory
AA_VARIANTS = {"aa_f32": "f32", "aa_f16": "f16"}
BYTES_PER_LUP.update({"aa_f32": 216, "aa_f16": 108})
# adjoint step: state gather + lambda(t+1) read + lambda(t) write (+ force read, force-gradient update)
ADJ_BYTES_PER_LUP = {"adjoint_f32": 108 + 108 + 108 + 12 + 24, "adjoint_f32_hbm": 108 + 108 + 108 + 12 + 24,
                     "adjoint_f16": 54 + 108 + 108,
                     # full corrections: the density pass (state read, density written), the adjoint step
                     # (as above plus the density read and the gradient cotangent written), the stencil's
                     # transpose (cotangent read, the node's 27 adjoint values read and written)
                     "adjoint_full_f32": (108 + 4) + (108 + 108 + 108 + 12 + 24 + 4 + 12) + (12 + 108 + 108),
                     # lagged time level: the density field comes from the forward run (no density pass),
                     # and the transpose of the previous call's cotangent is one value per node (cotangent
                     # read, value written) that the adjoint step reads and adds to the node's outputs
                     "adjoint_full_lagged_f32": (12 + 4) + (108 + 108 + 108 + 12 + 24 + 4 + 12 + 4)}
# forward step bytes of the state type an adjoint variant recomputes with (per-node force read included;
# the full corrections' exact time level adds a density pass and the density read)
ADJ_FORWARD_BYTES = {"adjoint_f32": 216 + 12, "adjoint_f32_hbm": 216 + 12, "adjoint_f16": 108,
                     "adjoint_full_f32": (108 + 4) + 216 + 12 + 4,
                     "adjoint_full_lagged_f32": 216 + 12 + 4 + 4}
# the paper's only cost figures (Sec. 6, shallow cavity, no hardware or times): node-count ratios cubic / cuboid
PAPER_CONTEXT = {"source": "Sec. 6 shallow lid-driven cavity, L/H = 4, W/H = 2, Re = 100; no hardware, precision or "
                           "times are given",
                 "cubic_over_cuboid_nodes": {"r=0.406,s=1.3": 7.88, "r=0.375,s=0.75": 5.33, "r=0.375,s=1.0": 7.11}}
KERNEL_SOURCES = ("paper_2107_14774_amd/csrc/lbm_device.h", "paper_2107_14774_amd/csrc/lbm_step.h",
                  "paper_2107_14774_amd/csrc/lbm_api.hip", "paper_2107_14774_amd/csrc/lbm_forward.hip")
ADJOINT_SOURCES = ("paper_2107_14774_amd/csrc/lbm_device.h", "paper_2107_14774_amd/csrc/lbm_adjoint_step.h",
                   "paper_2107_14774_amd/csrc/lbm_api.hip", "paper_2107_14774_amd/csrc/lbm_adjoint.hip")


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def sources_sha(paths):
    """Hash of the kernel sources without comments and whitespace runs (a comment edit leaves the
    profiled kernels, and so their measured traffic, unchanged)."""
    h = hashlib.sha256()
    for p in paths:
        with open(os.path.join(ROOT, p), encoding="utf-8") as fh:
            text = fh.read()
        text = re.sub(r"/\*.*?\*/", " ", text, flags=re.S)
        text = re.sub(r"//[^\n]*", " ", text)
        h.update(" ".join(text.split()).encode())
    return h.hexdigest()[:16]


def measured_traffic(kind):
    """HBM bytes per launch from profiles/traffic.json if it matches the current sources."""
    path = os.path.join(ROOT, "profiles", "traffic.json")
    if not os.path.exists(path):
        return None
    with open(path) as fh:
        rec = json.load(fh)
    entry = rec.get(kind)
    if not entry:
        return None
    srcs = ADJOINT_SOURCES if kind.startswith("adjoint") else KERNEL_SOURCES
    if entry.get("source_sha") != sources_sha(srcs):
        return None
    return entry.get("bytes_per_launch")


def time_steps(lat, a, b, steps, warmup, force=None, full_mode=None):
    """Warm up, then time exactly `steps` launches; returns (wall s, event ms per step, a, b).
    With ``full_mode`` the full corrections run through lbm_step_full (density fields allocated here)."""
    import paper_2107_14774_amd as P
    if full_mode is not None:
        da, db = lat.density(a), lat.field(1)
    if warmup:
        if full_mode is None:
            a, b = lat.step(a, b, warmup, force)
        else:
            a, b, da, db = lat.step_full(a, b, warmup, da, db, full_mode, force)
    torch.cuda.synchronize()
    stream = torch.cuda.current_stream()
    ev0, ev1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    t0 = time.perf_counter()
    ev0.record(stream)
    if full_mode is None:
        P.lbm_step(lat.h, steps, a, None if lat.aa else b, force, stream=stream)
    else:
        P.lbm_step_full(lat.h, steps, a, b, da, db, full_mode, force, stream=stream)
    ev1.record(stream)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    if steps % 2 and not lat.aa:
        a, b = b, a
    return wall, ev0.elapsed_time(ev1) / steps, a, b


def run_forward(w, variant, steps, warmup, u0_dev):
    import paper_2107_14774_amd as P
    storage, mode = FULL_VARIANTS.get(variant, (AA_VARIANTS.get(variant, variant), None))
    layout = "aa" if variant in AA_VARIANTS else "ab"
    if layout == "aa":  # the in-place layout advances in pairs of steps
        steps += steps % 2
        warmup += warmup % 2
    on, ox = P.relaxation_rates(w.nu, w.xi, w.cs2)
    lat = P.Lattice(w.nx, w.ny, w.nz, r=w.r, s=w.s, cs2=w.cs2, omega_nu=on, omega_xi=ox,
                    bc_y=w.bc_y, bc_z=w.bc_z, storage=storage, corr="local" if mode is None else "full", layout=layout)
    a, b = lat.new_state(), (None if layout == "aa" else lat.new_state())
    lat.init(a, u=u0_dev)
    torch.cuda.synchronize()
    log(f"[bench] {variant}: {w.nx}x{w.ny}x{w.nz}, state {lat.h.state_bytes / 2**30:.2f} GiB, "
        f"{warmup} warmup + {steps} timed steps")
    wall, ms_launch, a, b = time_steps(lat, a, b, steps, warmup, full_mode=mode)
    m = lat.moments(a)
    sums = P.lbm_check_sums(m.sums)
    mlups = lat.n * steps / wall / 1e6
    kernel_mlups = lat.n / (ms_launch * 1e-3) / 1e6
    log(f"[bench] {variant}: {mlups:.0f} MLUPS wall, {kernel_mlups:.0f} MLUPS per step "
        f"({ms_launch:.3f} ms/step), mass {sums[0]:.6f}, energy {sums[4]:.6e}")
    del a, b, lat
    torch.cuda.empty_cache()
    return {"mlups": mlups, "wall_s": wall, "ms_per_launch": ms_launch, "kernel_mlups": kernel_mlups,
            "mass": sums[0], "energy": sums[4]}


def copy_bandwidth(nbytes, reps=10):
    """Read+write GB/s of the library's plain copy (lbm_copy: one 16-byte non-temporal load and store per
    thread) of nbytes, timed with HIP events on the launch stream."""
    import paper_2107_14774_amd as P
    a = torch.empty(nbytes // 4, dtype=torch.float32, device="cuda").fill_(1.0)
    b = torch.empty_like(a)
    stream = torch.cuda.current_stream()
    P.lbm_copy(b, a, stream=stream)
    P.lbm_copy(b, a, stream=stream)
    torch.cuda.synchronize()
    ev0, ev1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    ev0.record(stream)
    for _ in range(reps):
        P.lbm_copy(b, a, stream=stream)
    ev1.record(stream)
    torch.cuda.synchronize()
    ms = ev0.elapsed_time(ev1) / reps
    del a, b
    torch.cuda.empty_cache()
    gbs = 2 * nbytes / (ms * 1e-3) / 1e9
    log(f"[bench] lbm_copy of {nbytes / 2**30:.2f} GiB: {ms:.3f} ms, {gbs:.0f} GB/s (read + write)")
    return gbs


def stream_bandwidth(w, steps, warmup, storage="f32"):
    """Streaming only (lbm_stream) on the workload's grid: the step's bytes in the step's access pattern and
    launch shape, without the collision.  Returns (GB/s at the step's algorithmic bytes, ms per launch)."""
    import paper_2107_14774_amd as P
    on, ox = P.relaxation_rates(w.nu, w.xi, w.cs2)
    lat = P.Lattice(w.nx, w.ny, w.nz, r=w.r, s=w.s, cs2=w.cs2, omega_nu=on, omega_xi=ox,
                    bc_y=w.bc_y, bc_z=w.bc_z, storage=storage, corr="local")
    a, b = lat.new_state(), lat.new_state()
    lat.init(a)
    stream = torch.cuda.current_stream()
    P.lbm_stream(lat.h, warmup + warmup % 2, a, b, stream=stream)
    torch.cuda.synchronize()
    ev0, ev1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    ev0.record(stream)
    P.lbm_stream(lat.h, steps, a, b, stream=stream)
    ev1.record(stream)
    torch.cuda.synchronize()
    ms = ev0.elapsed_time(ev1) / steps
    gbs = BYTES_PER_LUP[storage] * lat.n / (ms * 1e-3) / 1e9
    log(f"[bench] lbm_stream ({storage}, streaming only): {ms:.4f} ms per launch, {gbs:.0f} GB/s")
    del a, b, lat
    torch.cuda.empty_cache()
    return gbs, ms


def adjoint_workload(kind):
    """(workload, storage) of an adjoint variant: the C4 duct (128x128x64, FP32 state, per-node force; its
    working set is partly held by the 256 MB Infinity Cache), the same duct physics on 512x512x128 (3.6 GB
    state, HBM-resident), and the C5 periodic grid (384x384x192, FP16 state, initial-velocity gradient)."""
    if kind == "adjoint_f32":
        return W.ADJOINT_DUCT_128, "f32"
    if kind == "adjoint_f32_hbm":
        return W.replica(W.ADJOINT_DUCT_128, 512, 512, 128, name="adjoint_duct_512x512x128"), "f32"
    if kind in ("adjoint_full_f32", "adjoint_full_lagged_f32"):
        return W.replica(W.ADJOINT_DUCT_128, 512, 512, 128, name="adjoint_duct_512x512x128_full"), "f32"
    return W.ADJOINT_F16_384, "f16"


def run_adjoint(kind, steps, warmup):
    """Adjoint step kernel alone (repeated on one state), then one full backward pass of the workload's own
    trajectory length (recomputation of the checkpoint segments included)."""
    import paper_2107_14774_amd as P
    from paper_2107_14774_amd import adjoint as ADJ
    w, storage = adjoint_workload(kind)
    full = kind in ("adjoint_full_f32", "adjoint_full_lagged_f32")
    mode = "lagged" if kind == "adjoint_full_lagged_f32" else "exact"
    on, ox = P.relaxation_rates(w.nu, w.xi, w.cs2)
    lat = P.Lattice(w.nx, w.ny, w.nz, r=w.r, s=w.s, cs2=w.cs2, omega_nu=on, omega_xi=ox,
                    bc_y=w.bc_y, bc_z=w.bc_z, storage=storage, corr="full" if full else "local")
    force = None
    if storage == "f32":
        force = torch.from_numpy(W.body_force_field(w)).to(torch.float32).cuda()
        u0 = torch.zeros((3, w.nz, w.ny, w.nx), dtype=torch.float64, device="cuda")
    else:
        u0 = torch.from_numpy(W.initial_velocity(w)).cuda()
    st, tmp = lat.new_state(), lat.new_state()
    lat.init(st, u=u0)
    if full:
        drho, gwork, gpend = lat.field(1), lat.field(3), lat.field(3).zero_()
        st, tmp, _, _ = lat.step_full(st, tmp, 10, drho, None, "exact", force)
    else:
        st, tmp = lat.step(st, tmp, 10, force)
    lam_a = lat.new_adjoint().normal_()
    lam_b = lat.new_adjoint()
    grad = torch.zeros((3, w.nz, w.ny, w.nx), dtype=torch.float32, device="cuda") if force is not None else None
    stream = torch.cuda.current_stream()

    def adjoint_step(la, lb):
        nonlocal gwork, gpend
        if full and mode == "lagged":  # adjoint step, the transpose of the pending cotangent
            P.lbm_step_adjoint_full(lat.h, st, la, lb, drho, gwork, force, grad, mode="lagged", grad_pending=gpend,
                                    stream=stream)
            gwork, gpend = gpend, gwork
        elif full:  # density pass, adjoint step, the stencil's transpose
            P.lbm_step_adjoint_full(lat.h, st, la, lb, drho, gwork, force, grad, stream=stream)
        else:
            P.lbm_step_adjoint(lat.h, st, la, lb, force, grad, stream=stream)

    for _ in range(warmup):
        adjoint_step(lam_a, lam_b)
        lam_a, lam_b = lam_b, lam_a
    torch.cuda.synchronize()
    ev0, ev1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    ev0.record(stream)
    for _ in range(steps):
        adjoint_step(lam_a, lam_b)
        lam_a, lam_b = lam_b, lam_a
    ev1.record(stream)
    torch.cuda.synchronize()
    ms = ev0.elapsed_time(ev1) / steps
    mlups = lat.n / (ms * 1e-3) / 1e6
    alg = ADJ_BYTES_PER_LUP[kind] * lat.n / (ms * 1e-3) / 1e9
    pattern_gbs = None
    if not full:  # the same bytes in the adjoint step's access pattern without its arithmetic
        for _ in range(warmup):
            P.lbm_adjoint_stream(lat.h, st, lam_a, lam_b, force, grad, stream=stream)
            lam_a, lam_b = lam_b, lam_a
        torch.cuda.synchronize()
        ev0.record(stream)
        for _ in range(steps):
            P.lbm_adjoint_stream(lat.h, st, lam_a, lam_b, force, grad, stream=stream)
            lam_a, lam_b = lam_b, lam_a
        ev1.record(stream)
        torch.cuda.synchronize()
        pattern_gbs = ADJ_BYTES_PER_LUP[kind] * lat.n / (ev0.elapsed_time(ev1) / steps * 1e-3) / 1e9
        log(f"[bench] {kind}: lbm_adjoint_stream (the adjoint step's data movement only) {pattern_gbs:.0f} GB/s")
    del st, tmp, lam_a, lam_b, grad
    if full:
        del drho, gwork, gpend
    torch.cuda.empty_cache()
    # full backward passes over the workload's trajectory; the second is timed, so the recomputation
    # buffers come from the allocator's cache as in a training loop
    nsteps, every = w.steps, w.extra["checkpoint"]
    target = torch.zeros((3, w.nz, w.ny, w.nx), dtype=torch.float64, device="cuda")
    for rep in range(2):
        uc = u0.clone().requires_grad_(storage == "f16")
        Fc = force.clone().requires_grad_(True) if force is not None else None
        uT = ADJ.simulate(lat, uc, Fc, nsteps, every, full_mode=mode)
        loss = 0.5 * ((uT.to(torch.float64) - target) ** 2).sum()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        loss.backward()
        torch.cuda.synchronize()
        bwd = time.perf_counter() - t0
        del uT, loss, uc, Fc
    # algorithmic bytes of the backward: every adjoint step, plus the forward steps that recompute each
    # checkpoint segment (all but its first state); at the exact level of the full corrections the
    # recomputed steps leave each state's density behind, so only the adjoint step of a segment's last
    # state runs the density pass (112 B/LUP)
    nseg = -(-nsteps // every)
    recomputed = nsteps - nseg
    adj_bytes = ADJ_BYTES_PER_LUP[kind] * nsteps
    if kind == "adjoint_full_f32":
        adj_bytes -= (108 + 4) * (nsteps - nseg)
    bwd_bytes = (adj_bytes + ADJ_FORWARD_BYTES[kind] * recomputed) * lat.n
    bwd_gbs = bwd_bytes / bwd / 1e9
    log(f"[bench] {kind}: {w.nx}x{w.ny}x{w.nz} {storage}: adjoint step {ms:.3f} ms, {mlups:.0f} MLUPS, "
        f"{alg:.0f} GB/s algorithmic; backward of {nsteps} steps (checkpoint {every}) {bwd:.3f} s "
        f"= {lat.n * nsteps / bwd / 1e6:.0f} MLUPS, {bwd_gbs:.0f} GB/s incl. recomputation")
    n_nodes = lat.n
    del lat
    torch.cuda.empty_cache()
    return {"workload": w.name, "storage": storage, "mlups": round(mlups, 1), "ms_per_step": round(ms, 4),
            "hbm_gbs_algorithmic": round(alg, 1), "hbm_frac": round(alg / HBM_PEAK_GBS, 4),
            "pattern_ceiling_gbs": None if pattern_gbs is None else round(pattern_gbs, 1),
            "frac_of_pattern": None if pattern_gbs is None else round(alg / pattern_gbs, 4),
            "bytes_per_lup": ADJ_BYTES_PER_LUP[kind], "measured_bytes_per_launch": measured_traffic(kind),
            "backward_mlups_incl_recompute": round(n_nodes * nsteps / bwd / 1e6, 1),
            "backward_hbm_gbs_algorithmic": round(bwd_gbs, 1),
            "backward_hbm_frac": round(bwd_gbs / HBM_PEAK_GBS, 4),
            "backward_steps": nsteps, "checkpoint_every": every, "recomputed_forward_steps": recomputed}


def lat_n(w):
    return w.nx * w.ny * w.nz


def cpu_baseline(w):
    """The FP64 oracle (test infrastructure, untuned) on the host: 24 steps of a 64x64x32 replica of the
    workload (same r, s, viscosity and |k| <= 8 spectrum) on all host cores, 200 steps of the 32x32x16
    Taylor-Green configuration on all cores, and 2 replica steps on one thread (about 20 s in all)."""
    import oracle
    from oracle import analytic as A
    from oracle import lbm as OL
    cores = len(os.sched_getaffinity(0))
    torch.set_num_threads(cores)

    def oracle_run(rep, u0, steps):
        p = oracle.Params(rep.nx, rep.ny, rep.nz, r=rep.r, s=rep.s, cs2=rep.cs2,
                          omega_nu=A.omega_from_nu(rep.nu, rep.cs2), omega_xi=A.omega_from_xi(rep.xi, rep.cs2),
                          corr="local")
        f = OL.init_equilibrium(torch.ones(p.shape, dtype=torch.float64), torch.as_tensor(u0), p)
        f = OL.step(f, p)
        t0 = time.perf_counter()
        for _ in range(steps):
            f = OL.step(f, p)
        dt = time.perf_counter() - t0
        return p.n * steps / dt / 1e6, dt

    rep = W.replica(w, 64, 64, 32)
    u_rep = W.initial_velocity(rep)
    steps = 24
    val, dt = oracle_run(rep, u_rep, steps)
    used = torch.get_num_threads()
    log(f"[bench] cpu oracle: {val:.4f} MLUPS on {used} threads, {rep.nx}x{rep.ny}x{rep.nz} replica ({dt:.1f} s)")
    c1 = W.TAYLOR_GREEN_32
    val_c1, dt_c1 = oracle_run(c1, W.initial_velocity(c1), c1.steps)
    log(f"[bench] cpu oracle: {val_c1:.4f} MLUPS on {used} threads, {c1.name} {c1.steps} steps ({dt_c1:.1f} s)")
    torch.set_num_threads(1)
    steps1 = 2
    val1, dt1 = oracle_run(rep, u_rep, steps1)
    torch.set_num_threads(cores)
    log(f"[bench] cpu oracle: {val1:.4f} MLUPS on 1 thread ({dt1:.1f} s)")
    return {"value": val, "unit": "MLUPS", "cores": used, "kind": "oracle",
            "sample": f"FP64 oracle, {steps} steps of the {rep.nx}x{rep.ny}x{rep.nz} replica of the workload "
                      f"(r={rep.r}, s={rep.s}, same viscosity, |k| <= {rep.extra['kmax']} modes), {dt:.1f} s",
            "taylor_green_32x32x16_value": val_c1,
            "taylor_green_32x32x16_sample": f"{c1.steps} steps of {c1.name} on {used} threads, {dt_c1:.1f} s",
            "single_thread_value": val1,
            "single_thread_sample": f"{steps1} steps of the replica on 1 thread, {dt1:.1f} s"}


# ---------------------------------------------------------------------- rocprofv3 summaries
PROFILE_KERNELS = {
    "f32": "k_step<0, 2, 0, false, false>", "f16": "k_step_pair<1, 2, false, false>",
    "bf16": "k_step_pair<2, 2, false, false>", "bf16_sr": "k_step_pair<3, 2, false, false>",
    "full_f32": "k_step<0, 3, 0, false, false>", "full_f16": "k_step_full_pair<1, false>",
    "aa_f32 (local)": "k_step_aa<0, 2, false, false, false, false>", "aa_f32 (shifted)": "k_step_aa<0, 2, true, false, false, false>",
    "aa_f16 (local)": "k_step_aa_pair<1, 2, false, false, false, false>",
    "aa_f16 (shifted)": "k_step_aa_pair<1, 2, true, false, false, true>",
    "adjoint_f32": "k_step_adjoint<0, 2, 1, false, false>", "adjoint_f32_hbm": "k_step_adjoint<0, 2, 1, false, false>",
    "adjoint_f16": "k_step_adjoint<1, 2, 0, false, false>",
    # the adjoint of the full corrections: its step kernel and the stencil's transpose added to the 27
    # adjoint values of every node (exact time level), or written as one value per node that the next
    # adjoint step adds (lagged); the density pass is k_density, shared with the recomputed forward steps
    "adjoint_full (step)": "k_step_adjoint<0, 3, 1, false, false>",
    "adjoint_full (transpose)": "k_density_vjp<false>", "adjoint_full (lagged transpose)": "k_density_vjp<true>",
    # the measured ceilings: streaming only (the FP32 step and the FP16 pair step without their
    # collisions) and the plain copy
    "stream_f32": "k_stream<0, 0>", "stream_f16": "k_stream_pair<1>", "copy": "k_copy16",
    # and the adjoint step's data movement without its arithmetic, on the adjoint workloads
    "adjoint_stream_f32": "k_adjoint_stream<0, 1>", "adjoint_stream_f32_hbm": "k_adjoint_stream<0, 1>",
    "adjoint_stream_f16": "k_adjoint_stream<1, 0>",
}
PROFILE_WORKLOADS = {  # variant -> (nx, ny, nz, label)
    "f32": (512, 512, 256, "512x512x256"), "f16": (512, 512, 256, "512x512x256"),
    "bf16": (512, 512, 256, "512x512x256"), "bf16_sr": (512, 512, 256, "512x512x256"),
    "full_f32": (512, 512, 256, "512x512x256"),
    "full_f16": (512, 512, 256, "512x512x256"), "adjoint_f32": (128, 128, 64, "128x128x64 duct"),
    "aa_f32 (local)": (512, 512, 256, "512x512x256"), "aa_f32 (shifted)": (512, 512, 256, "512x512x256"),
    "aa_f16 (local)": (512, 512, 256, "512x512x256"), "aa_f16 (shifted)": (512, 512, 256, "512x512x256"),
    "adjoint_f16": (384, 384, 192, "384x384x192"), "adjoint_f32_hbm": (512, 512, 128, "512x512x128 duct"),
    "adjoint_full (step)": (512, 512, 128, "512x512x128 duct"),
    "adjoint_full (transpose)": (512, 512, 128, "512x512x128 duct"),
    "adjoint_full (lagged transpose)": (512, 512, 128, "512x512x128 duct"),
    "stream_f32": (512, 512, 256, "512x512x256"), "stream_f16": (512, 512, 256, "512x512x256"),
    "copy": (512, 512, 256, "one FP32 state"),
    "adjoint_stream_f32": (128, 128, 64, "128x128x64 duct"),
    "adjoint_stream_f32_hbm": (512, 512, 128, "512x512x128 duct"),
    "adjoint_stream_f16": (384, 384, 192, "384x384x192"),
}
COPY_BYTES = 27 * 512 * 512 * 256 * 4                 # bytes read (and written) by one lbm_copy of the bench
# $OUT is any output directory (the three runs write their CSVs under it)
TRACE_CMD = ("rocprofv3 --kernel-trace --stats -d $OUT/prof_step -o step --output-format csv -- "
             "python3 bench.py --steps 30 --warmup 5 --no-cpu-baseline")
PMC_CMD = ("timeout -s KILL 600 rocprofv3 --pmc {c} -d $OUT/pmc_{d} -o {d} --output-format csv -- "
           "python3 bench.py --steps 4 --warmup 1 --no-cpu-baseline")
SUMMARY_CMD = "python3 bench.py --summarize-rocprof $OUT"
TRACE_SUMMARY = "profiles/k_step_and_adjoint_kernel_trace.txt"
TRAFFIC_SUMMARY = "profiles/k_step_and_adjoint_hbm_traffic.txt"
VALU_COUNTERS = "VALUBusy SQ_INSTS_VALU SQ_WAVES"
VALU_SUMMARY = "profiles/k_step_and_adjoint_valu_busy.txt"


def _launch_grid(nx, ny, nz, kernel=""):
    """Total threads of a node-kernel launch (the library's block-width rule; the 16-bit
    two-nodes-per-thread kernels run nx / 2 threads per row in blocks of 128)."""
    if "_pair<" in kernel:
        return str((nx // 2 + 127) // 128 * 128 * ny * nz)
    if kernel == "k_copy16":
        return str((COPY_BYTES // 16 + 255) // 256 * 256)
    best, waste = 256, 1 << 30
    for b in (256, 192, 128, 64):
        w = (nx + b - 1) // b * b - nx
        if w < waste:
            best, waste = b, w
    return str((nx + best - 1) // best * best * ny * nz)


def summarize_rocprof(out_dir):
    """Write the kernel-trace and HBM-traffic summaries (and traffic.json) under profiles/ from the
    CSVs of the three rocprofv3 runs named in TRACE_CMD and PMC_CMD, found under ``out_dir``."""
    import csv
    import statistics
    alg = dict(BYTES_PER_LUP, **ADJ_BYTES_PER_LUP)
    for v in PROFILE_KERNELS:
        if v.startswith("aa_"):
            alg[v] = BYTES_PER_LUP[v.split()[0]]
    alg["stream_f32"] = BYTES_PER_LUP["f32"]
    alg["stream_f16"] = BYTES_PER_LUP["f16"]
    for v in ("adjoint_stream_f32", "adjoint_stream_f32_hbm", "adjoint_stream_f16"):
        alg[v] = ADJ_BYTES_PER_LUP[v.replace("_stream", "")]
    alg["adjoint_full (step)"] = 108 + 108 + 108 + 12 + 24 + 4 + 12
    alg["adjoint_full (transpose)"] = 12 + 108 + 108
    alg["adjoint_full (lagged transpose)"] = 12 + 4
    alg["copy"] = 2 * COPY_BYTES // (512 * 512 * 256)   # per node of the state copied
    trace = list(csv.DictReader(open(os.path.join(out_dir, "prof_step", "step_kernel_trace.csv"))))
    lines = ["# rocprofv3 kernel trace: fused collide-and-stream step (512x512x256, r=1, s=1/2; local and full",
             "# corrections), its adjoint (128x128x64 and 512x512x128 ducts with force field; 384x384x192,",
             "# r=1/2, s=1/4, FP16), and the measured ceilings: streaming only (k_stream and k_stream_pair, the",
             "# FP32 and FP16 steps' gathers and stores without the collisions; k_adjoint_stream, the adjoint",
             "# step's loads and stores without its arithmetic) and the library copy (k_copy16, one FP32 state)",
             "", "commands (repo root, one MI355X, TMPDIR=/tmp, $OUT an output directory):", "  " + TRACE_CMD,
             "  " + SUMMARY_CMD, "",
             f"{'kernel':38s} {'variant':16s} {'workload':16s} calls  avg_ms   min_ms   max_ms   "
             "MLUPS(avg)  alg_B/LUP  alg_GB/s  frac_of_8TB/s"]
    for v, key in PROFILE_KERNELS.items():
        nx, ny, nz, label = PROFILE_WORKLOADS[v]
        grid = _launch_grid(nx, ny, nz, key)
        d = [int(r["End_Timestamp"]) - int(r["Start_Timestamp"]) for r in trace
             if key in r["Kernel_Name"] and r["Grid_Size_X"] == grid]
        if not d:
            continue
        n = nx * ny * nz
        avg = statistics.mean(d) / 1e6
        b = alg[v]
        lines.append(f"{key:38s} {v:16s} {label:16s} {len(d):5d}  {avg:.4f}  {min(d) / 1e6:.4f}  {max(d) / 1e6:.4f}"
                     f"  {n / avg / 1e3:10.0f}  {b:9d}  {b * n / avg / 1e6:8.0f}  {b * n / avg / 1e6 / HBM_PEAK_GBS:.3f}")
    lines += ["", "(kernels grouped by name and grid size; the adjoint calls include the backward passes of bench.py)"]
    with open(os.path.join(ROOT, TRACE_SUMMARY), "w") as fh:
        fh.write("\n".join(lines) + "\n")

    def rows(kind):
        return list(csv.DictReader(open(os.path.join(out_dir, f"pmc_{kind}", f"{kind}_counter_collection.csv"))))
    fe, wr = rows("fetch"), rows("write")
    copy_bytes = COPY_BYTES
    # the library copies of copy_bandwidth() (k_copy16 over one FP32 state) read and write known bytes
    cf = [float(r["Counter_Value"]) for r in fe if "k_copy16" in r["Kernel_Name"]]
    cw = [float(r["Counter_Value"]) for r in wr if "k_copy16" in r["Kernel_Name"]]
    kf = (copy_bytes / 1024) / statistics.mean(cf)
    kw = (copy_bytes / 1024) / statistics.mean(cw)
    lines = ["# HBM traffic of the step kernels (512x512x256, r=1, s=1/2) and the adjoint from rocprofv3 counters",
             "", "commands (repo root, one MI355X, TMPDIR=/tmp, $OUT an output directory), one counter per pass:",
             "  " + PMC_CMD.format(c="FETCH_SIZE", d="fetch"), "  " + PMC_CMD.format(c="WRITE_SIZE", d="write"),
             "  " + SUMMARY_CMD, "",
             "calibration: the library copy in the same runs (k_copy16 over one FP32 state, reads and writes",
             f"exactly {copy_bytes} bytes, {len(cf)} launches): mean FETCH_SIZE {statistics.mean(cf):.1f} KiB -> "
             f"scale {kf:.4f};", f"mean WRITE_SIZE {statistics.mean(cw):.1f} KiB -> scale {kw:.4f}", "",
             f"{'kernel':38s} {'variant':16s} FETCH_KiB(raw)  WRITE_KiB(raw)  read_B/LUP  write_B/LUP  "
             "total_B/LUP  algorithmic_B/LUP"]
    traffic = {}
    for v, key in PROFILE_KERNELS.items():
        nx, ny, nz, _ = PROFILE_WORKLOADS[v]
        grid = _launch_grid(nx, ny, nz, key)
        fv = [float(r["Counter_Value"]) for r in fe if key in r["Kernel_Name"] and r["Grid_Size"] == grid]
        wv = [float(r["Counter_Value"]) for r in wr if key in r["Kernel_Name"] and r["Grid_Size"] == grid]
        if not fv or not wv:
            continue
        n = nx * ny * nz
        rb = statistics.mean(fv) * 1024 * kf / n
        wb = statistics.mean(wv) * 1024 * kw / n
        lines.append(f"{key:38s} {v:16s} {statistics.mean(fv):14.1f}  {statistics.mean(wv):14.1f}  {rb:10.2f}  "
                     f"{wb:11.2f}  {rb + wb:11.2f}  {alg[v]:17d}")
        traffic[v] = {"kernel": key, "bytes_per_launch": round((rb + wb) * n), "bytes_per_lup": round(rb + wb, 3),
                      "read_bytes_per_lup": round(rb, 3), "write_bytes_per_lup": round(wb, 3),
                      "source_sha": sources_sha(ADJOINT_SOURCES if v.startswith("adjoint") else KERNEL_SOURCES),
                      "summary": TRAFFIC_SUMMARY}
    with open(os.path.join(ROOT, TRAFFIC_SUMMARY), "w") as fh:
        fh.write("\n".join(lines) + "\n")
    with open(os.path.join(ROOT, "profiles", "traffic.json"), "w") as fh:
        json.dump(traffic, fh, indent=1)
    print(open(os.path.join(ROOT, TRACE_SUMMARY)).read())
    print(open(os.path.join(ROOT, TRAFFIC_SUMMARY)).read())
    if os.path.isdir(os.path.join(out_dir, "pmc_valu")):
        summarize_valu(out_dir)


def summarize_valu(out_dir):
    """VALU summary from the optional third counter pass (VALU_COUNTERS): rocprofv3's derived
    VALUBusy (time the vector ALUs issue, % of the kernel's GPU time) and the executed VALU
    instructions per wave, per profiled kernel."""
    import csv
    import statistics
    rows = list(csv.DictReader(open(os.path.join(out_dir, "pmc_valu", "valu_counter_collection.csv"))))
    lines = ["# VALU activity of the step kernels (512x512x256, r=1, s=1/2) and the adjoint from rocprofv3 counters",
             "", "commands (repo root, one MI355X, TMPDIR=/tmp, $OUT an output directory):",
             "  " + PMC_CMD.format(c=VALU_COUNTERS, d="valu"), "  " + SUMMARY_CMD, "",
             "VALUBusy = 100 * sum(SQ_ACTIVE_INST_VALU) / CU_NUM / GRBM_GUI_ACTIVE (rocprofv3's definition for",
             "gfx950); VALU/wave = SQ_INSTS_VALU / SQ_WAVES (executed, so exits and branches count as run).", "",
             f"{'kernel':44s} {'variant':16s} dispatches  VALUBusy_%  VALU/wave"]
    for v, key in PROFILE_KERNELS.items():
        nx, ny, nz, _ = PROFILE_WORKLOADS[v]
        grid = _launch_grid(nx, ny, nz, key)
        mine = [r for r in rows if key in r["Kernel_Name"] and r["Grid_Size"] == grid]
        if not mine:
            continue
        busy = [float(r["Counter_Value"]) for r in mine if r["Counter_Name"] == "VALUBusy"]
        insts = [float(r["Counter_Value"]) for r in mine if r["Counter_Name"] == "SQ_INSTS_VALU"]
        waves = [float(r["Counter_Value"]) for r in mine if r["Counter_Name"] == "SQ_WAVES"]
        if not busy or not insts or not waves:
            continue
        lines.append(f"{key:44s} {v:16s} {len(busy):10d}  {statistics.mean(busy):10.1f}  "
                     f"{sum(insts) / sum(waves):9.0f}")
    with open(os.path.join(ROOT, VALU_SUMMARY), "w") as fh:
        fh.write("\n".join(lines) + "\n")
    print(open(os.path.join(ROOT, VALU_SUMMARY)).read())


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=200)
    ap.add_argument("--warmup", type=int, default=20)
    ap.add_argument("--variants", default="f32,f16,bf16,bf16_sr,full_f32,full_f16,aa_f32,aa_f16,adjoint_f32,"
                                          "adjoint_f32_hbm,adjoint_f16,adjoint_full_f32,adjoint_full_lagged_f32")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--summarize-rocprof", metavar="DIR", default=None,
                    help="write the profiles/ summaries from rocprofv3 CSVs under DIR (no GPU needed)")
    args = ap.parse_args()
    if args.summarize_rocprof:
        summarize_rocprof(args.summarize_rocprof)
        return
    if args.gpus != 1:
        print(f"bench.py measures one GPU only: --gpus {args.gpus} is not supported "
              "(the multi-GPU z-slab decomposition is a design note, not built)", file=sys.stderr)
        sys.exit(2)
    if not torch.cuda.is_available():
        print("bench.py needs a GPU", file=sys.stderr)
        sys.exit(2)
    torch.cuda.set_device(0)
    w = W.DECAYING_512
    variants = [v for v in args.variants.split(",") if v]
    log(f"[bench] generating the initial velocity field ({w.nx}x{w.ny}x{w.nz})")
    u0_dev = torch.from_numpy(W.initial_velocity(w)).to("cuda")

    state_bytes = 27 * w.nx * w.ny * w.nz * 4          # one FP32 state (rows already whole blocks)
    copy_gbs = copy_bandwidth(state_bytes)
    pattern_gbs, pattern_ms = stream_bandwidth(w, max(20, args.steps // 4), args.warmup)
    pattern16 = None
    if any(v in ("f16", "bf16", "bf16_sr") for v in variants):   # the 16-bit steps' own pattern
        pattern16 = stream_bandwidth(w, max(20, args.steps // 4), args.warmup, "f16")
    res = {}
    for v in variants:
        if v in BYTES_PER_LUP:
            res[v] = run_forward(w, v, args.steps, args.warmup, u0_dev)
    del u0_dev
    torch.cuda.empty_cache()
    adj = {}
    for v in variants:
        if v in ADJ_BYTES_PER_LUP:
            adj[v] = run_adjoint(v, max(20, args.steps // 4), 3)

    variants_out = {}
    roofline = None
    r = None
    main_v = None
    if res:
        main_v = "f32" if "f32" in res else next(iter(res))
        main_storage, main_mode = FULL_VARIANTS.get(main_v, (main_v, None))
        r = res[main_v]
        achieved = BYTES_PER_LUP[main_v] * (w.n) / (r["ms_per_launch"] * 1e-3) / 1e9
        roofline = {"bound": "hbm", "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
                    "frac": round(achieved / HBM_PEAK_GBS, 4), "traffic": measured_traffic(main_v),
                    "kernel": f"k_step<{main_storage}, {'local' if main_mode is None else 'full'} corrections>",
                    "algorithmic_bytes_per_lup": BYTES_PER_LUP[main_v],
                    "device_copy_gbs": round(copy_gbs, 1), "frac_of_copy": round(achieved / copy_gbs, 4),
                    "copy": "lbm_copy of one FP32 state, 16 B per thread, non-temporal",
                    "pattern_ceiling_gbs": round(pattern_gbs, 1), "frac_of_pattern": round(achieved / pattern_gbs, 4),
                    "pattern": "lbm_stream: the FP32 step's gather and store without the collision, same launch "
                               f"shape ({pattern_ms:.4f} ms per launch)"}
    for v, rv in res.items():
        ach = BYTES_PER_LUP[v] * w.n / (rv["ms_per_launch"] * 1e-3) / 1e9
        variants_out[v] = {"mlups": round(rv["mlups"], 1), "ms_per_step": round(rv["wall_s"] / args.steps * 1e3, 4),
                           "hbm_gbs_algorithmic": round(ach, 1), "hbm_frac": round(ach / HBM_PEAK_GBS, 4),
                           "bytes_per_lup": BYTES_PER_LUP[v], "measured_bytes_per_launch": measured_traffic(v)}
        if v in ("f16", "bf16", "bf16_sr") and pattern16:
            variants_out[v]["pattern_ceiling_gbs"] = round(pattern16[0], 1)
            variants_out[v]["frac_of_pattern"] = round(ach / pattern16[0], 4)
    variants_out.update(adj)
    if "f32" in res:
        for v in ("f16", "bf16", "bf16_sr", "full_f32", "full_f16", "full_f32_exact", "aa_f32", "aa_f16"):
            if v in res:
                variants_out[v]["speedup_vs_f32"] = round(res[v]["mlups"] / res["f32"]["mlups"], 3)

    line = {
        "metric": "MLUPS and % HBM roofline: plain FP32 vs BF16/FP16-storage vs adjoint",
        "value": round(r["mlups"], 1) if r else None,
        "unit": "MLUPS",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(r["wall_s"] / args.steps * 1e3, 4) if r else None,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": w.name, "nx": w.nx, "ny": w.ny, "nz": w.nz, "r": w.r, "s": w.s,
                   "cs2": w.cs2, "nu": w.nu, "corrections": "local", "boundaries": "periodic",
                   "storage": main_v or "none",
                   "fp32_conservation": "FP32 storage and arithmetic; each node's mass and momentum residual of "
                                        "the rounded outputs is summed in FP64 and put back (not in the paper)"},
        "paper_context": PAPER_CONTEXT,
        "roofline": roofline,
        "variants": variants_out,
    }
    if not args.no_cpu_baseline:
        line["cpu_baseline"] = cpu_baseline(w)
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
