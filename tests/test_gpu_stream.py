"""GPU checks of the measurement references: streaming only (the step's gather
and store without the collision) equals the oracle's streaming operator (Sec.
3.2, halfway bounce-back of Sec. 4 with stationary walls) bit for bit, since it
only moves stored values; the plain copy reproduces its source."""

import sys

import pytest
import torch

import oracle
from oracle import streaming as OS
from helpers import fp32_rounded_state, gpu_lattice, random_state

pytestmark = pytest.mark.gpu


def _say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


CASES = [
    # name, grid, (bc_x, bc_y, bc_z), storage
    ("periodic_ragged_f32", (300, 6, 5), ("periodic",) * 3, "f32"),
    ("duct_f32", (37, 12, 10), ("periodic", "bounceback", "bounceback"), "f32"),
    ("box_f16", (14, 10, 8), ("bounceback",) * 3, "f16"),
    ("periodic_bf16", (130, 5, 4), ("periodic",) * 3, "bf16"),
    ("duct_bf16_sr", (64, 8, 6), ("periodic", "bounceback", "bounceback"), "bf16_sr"),
    # even nx, periodic, 16-bit: the two-nodes-per-thread shape of the step
    ("periodic_f16_pairs", (258, 5, 3), ("periodic",) * 3, "f16"),
    ("periodic_bf16_sr_pairs", (130, 4, 5), ("periodic",) * 3, "bf16_sr"),
]


@pytest.mark.parametrize("case", CASES, ids=[c[0] for c in CASES])
def test_stream_only_equals_oracle_streaming(case):
    import paper_2107_14774_amd as P
    name, (nx, ny, nz), (bx, by, bz), storage = case
    _say("case", name)
    p = oracle.Params(nx, ny, nz, r=1.0, s=0.5, omega_nu=1.4, omega_xi=1.2, bc_x=bx, bc_y=by, bc_z=bz)
    lat = gpu_lattice(p, storage=storage)
    a, b = lat.new_state(), lat.new_state()
    lat.import_populations(a, fp32_rounded_state(random_state(p, 81), p).cuda())
    f = lat.export_populations(a).cpu()           # the stored values, as natural populations
    want = f
    for n in (1, 2):
        P.lbm_stream(lat.h, 1, a, b)
        a, b = b, a
        want = OS.stream(want, p)
        got = lat.export_populations(a).cpu()
        _say(f"{name}: after {n} streaming steps max |GPU - oracle| = {(got - want).abs().max().item():.3e}")
        assert torch.equal(got, want)


def test_copy_reproduces_source():
    import paper_2107_14774_amd as P
    g = torch.Generator(device="cuda").manual_seed(5)
    src = torch.rand(3 * 2**20 + 4, device="cuda", generator=g)     # 12 MiB + 16 B: one partial block
    dst = torch.zeros_like(src)
    P.lbm_copy(dst, src)
    torch.cuda.synchronize()
    assert torch.equal(dst, src)
    dst.zero_()
    P.lbm_copy(dst, src, 4096)                    # a prefix only
    torch.cuda.synchronize()
    assert torch.equal(dst[:1024], src[:1024]) and not dst[1024:].any()


ADJ_STREAM_CASES = [
    # name, grid, (bc_x, bc_y, bc_z), storage, per-node force, gather kind override
    ("periodic_f32_force", (300, 6, 5), ("periodic",) * 3, "f32", True, None),
    ("duct_f32_force", (37, 12, 10), ("periodic", "bounceback", "bounceback"), "f32", True, None),
    ("box_f16", (14, 10, 8), ("bounceback",) * 3, "f16", False, None),
    ("box_f32_64bit_slots", (14, 10, 8), ("bounceback",) * 3, "f32", True, "2"),
    ("periodic_bf16", (130, 5, 4), ("periodic",) * 3, "bf16", False, None),
]


@pytest.mark.parametrize("case", ADJ_STREAM_CASES, ids=[c[0] for c in ADJ_STREAM_CASES])
def test_adjoint_stream_moves_what_the_adjoint_step_reads(case):
    """lbm_adjoint_stream, the adjoint step's data movement: each node's output element b equals the
    population it gathered as f_b (the stored deviation) plus lambda(t+1) of what it emits in direction
    b, read where the adjoint step reads it (the downstream node's f_b, or across a wall the node's own
    f_opp(b)); force added to its gradient.  Exact in FP32."""
    import os
    import paper_2107_14774_amd as P
    from oracle import equilibrium as EQ
    from oracle import lattice as OLT
    name, (nx, ny, nz), (bx, by, bz), storage, field, kind = case
    _say("case", name)
    p = oracle.Params(nx, ny, nz, r=1.0, s=0.5, omega_nu=1.4, omega_xi=1.2, bc_x=bx, bc_y=by, bc_z=bz)
    old = os.environ.get("LBM_GATHER_KIND")
    if kind:
        os.environ["LBM_GATHER_KIND"] = kind
    try:
        lat = gpu_lattice(p, storage=storage)
    finally:
        if old is None:
            os.environ.pop("LBM_GATHER_KIND", None)
        else:
            os.environ["LBM_GATHER_KIND"] = old
    st = lat.new_state()
    lat.import_populations(st, fp32_rounded_state(random_state(p, 83), p).cuda())
    f = lat.export_populations(st).cpu()
    w = EQ.rest_weights(p.r, p.s, p.cs2)[:, None, None, None]
    dev = (f - w).to(torch.float32)                   # what the kernels gather (exact: see the export)
    g = torch.Generator().manual_seed(84)
    lam = torch.randn((27, nz, ny, nx), generator=g, dtype=torch.float64).to(torch.float32)
    lam_in, lam_out = lat.new_adjoint(), lat.new_adjoint()
    P.lbm_adjoint_from_natural(lat.h, lam.to(torch.float64).cuda(), lam_in)
    force = torch.randn((3, nz, ny, nx), generator=g).to(torch.float32) if field else None
    gF0 = torch.randn((3, nz, ny, nx), generator=g).to(torch.float32)
    gF = gF0.cuda() if field else None
    P.lbm_adjoint_stream(lat.h, st, lam_in, lam_out, None if force is None else force.cuda(), gF)
    got = torch.empty((27, nz, ny, nx), dtype=torch.float64, device="cuda")
    P.lbm_adjoint_to_natural(lat.h, lam_out, got)
    got = got.cpu()
    eb, opp = OLT.ebar(), OLT.opposite()
    walls = (bz == "bounceback", by == "bounceback", bx == "bounceback")
    idx = [torch.arange(n) for n in (nz, ny, nx)]
    want = torch.empty((27, nz, ny, nx), dtype=torch.float32)
    for b in range(27):
        e = (int(eb[b, 2]), int(eb[b, 1]), int(eb[b, 0]))          # (z, y, x)
        shifted = torch.roll(lam[b], shifts=tuple(-v for v in e), dims=(0, 1, 2))
        out = torch.zeros((nz, ny, nx), dtype=torch.bool)
        for d in range(3):
            if walls[d] and e[d] != 0:
                beyond = (idx[d] + e[d] < 0) | (idx[d] + e[d] >= (nz, ny, nx)[d])
                shape = [1, 1, 1]
                shape[d] = -1
                out |= beyond.reshape(shape).expand(nz, ny, nx)
        want[b] = dev[b] + torch.where(out, lam[opp[b]], shifted)
    err = (got - want.to(torch.float64)).abs().max().item()
    _say(f"{name}: max |got - want| = {err:.3e}")
    assert torch.equal(got, want.to(torch.float64))
    if field:
        assert torch.equal(gF.cpu(), gF0 + force)
