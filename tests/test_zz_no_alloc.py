"""The allocation-free adjoint step of the full corrections (lbm_step_adjoint_full_noalloc, static work
array) against lbm_step_adjoint_full at the exact time level with caller work fields: two calls in a
row on one device, the second on a smaller grid (the array keeps the first call's contents)."""

import sys

import numpy as np
import pytest
import torch

import oracle
import paper_2107_14774_amd as P
from helpers import fp32_rounded_state, gpu_lattice, random_state

pytestmark = pytest.mark.gpu

CASES = [
    # grid, r, s, (bc_x, bc_y, bc_z), storage, per-node force field
    ((40, 12, 10), 1.0, 0.5, ("periodic", "bounceback", "bounceback"), "f32", True),
    ((24, 8, 6), 0.5, 0.25, ("periodic",) * 3, "f16", False),
]


def _say(*a):
    print(*a)
    sys.stdout.flush()


def _outputs(lat, p, st, lam_in, force, noalloc):
    lam_out = lat.new_adjoint()
    gF = torch.zeros((3, *p.shape), dtype=torch.float32, device="cuda")
    gFu = torch.zeros(3, dtype=torch.float64, device="cuda")
    if noalloc:
        P.lbm_step_adjoint_full_noalloc(lat.h, st, lam_in, lam_out, force, gF, gFu)
    else:
        P.lbm_step_adjoint_full(lat.h, st, lam_in, lam_out, lat.field(1), lat.field(3), force, gF, gFu)
    torch.cuda.synchronize()
    return lam_out, gF, gFu


def test_noalloc_full_adjoint_matches_work_field_entry_point():
    for (nx, ny, nz), r, s, (bx, by, bz), storage, field in CASES:
        _say(f"no-alloc full adjoint: {nx}x{ny}x{nz} {storage} bc {bx}/{by}/{bz}")
        p = oracle.Params(nx, ny, nz, r=r, s=s, omega_nu=1.45, omega_xi=1.27, corr="full", bc_x=bx, bc_y=by,
                          bc_z=bz)
        lat = gpu_lattice(p, storage=storage)
        st = lat.new_state()
        lat.import_populations(st, fp32_rounded_state(random_state(p, 51), p).cuda())
        g = np.random.Generator(np.random.PCG64(52))
        lam_in = lat.new_adjoint()
        P.lbm_adjoint_from_natural(lat.h, torch.tensor(g.standard_normal((27, *p.shape))).cuda(), lam_in)
        force = torch.tensor(1e-4 * g.standard_normal((3, *p.shape))).to(torch.float32).cuda() if field else None
        got = _outputs(lat, p, st, lam_in, force, True)
        want = _outputs(lat, p, st, lam_in, force, False)
        # same kernels on the same inputs: the adjoint and the per-node force gradient bit for bit; the
        # uniform-force gradient sums block totals with atomics, in any order
        assert torch.equal(got[0], want[0])
        assert torch.equal(got[1], want[1])
        assert torch.allclose(got[2], want[2], rtol=1e-12, atol=0.0)
        _say(f"  max |lambda| {want[0].abs().max().item():.3e}: equal")
