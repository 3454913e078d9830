"""GPU checks of the AA layout (one buffer, in place): after an even number of
steps its state equals the two-buffer (AB) state bit for bit, since both gather
the same values and run the same collision; observables and time-dependent
forcing agree as well."""

import sys

import numpy as np
import pytest
import torch

import oracle
from helpers import fp32_rounded_state, gpu_lattice, random_state

pytestmark = pytest.mark.gpu
DT = torch.float64
Z3 = (0.0, 0.0, 0.0)


def _say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def _lattices(p, storage, force=Z3):
    import paper_2107_14774_amd as P
    kw = dict(r=p.r, s=p.s, cs2=p.cs2, omega_nu=p.omega_nu, omega_xi=p.omega_xi, omega_hi=p.omega_hi,
              bc_x=p.bc_x, bc_y=p.bc_y,
              bc_z=p.bc_z, storage=storage, corr=p.corr, force=force, wall_velocity=p.wall_velocity, moments=p.moments)
    return P.Lattice(p.nx, p.ny, p.nz, **kw), P.Lattice(p.nx, p.ny, p.nz, layout="aa", **kw)


CASES = [
    # name, grid, r, s, (bc_x, bc_y, bc_z), walls moving, corr, moments, storage, force field
    ("periodic_ragged_f32", (300, 6, 5), 1.0, 0.5, ("periodic",) * 3, None, "local", "central", "f32", False),
    ("duct_force_field_f32", (37, 12, 10), 1.0, 0.25, ("periodic", "bounceback", "bounceback"), None, "local",
     "central", "f32", True),
    ("cavity_moving_faces_f32", (14, 10, 8), 0.5, 1.0, ("bounceback",) * 3,
     ((0, 0, 0), (0, 0.01, 0), (0, 0, 0), (0.05, 0, 0.02), (0.03, 0, 0), (0, 0, 0)), "local", "central", "f32", False),
    ("periodic_f16_lowmach", (70, 9, 6), 0.5, 0.25, ("periodic",) * 3, None, "lowmach", "central", "f16", False),
    ("cavity_raw_bf16", (12, 16, 12), 0.75, 1.0, ("bounceback",) * 3,
     ((0, 0, 0),) * 3 + ((0.06, 0, 0),) + ((0, 0, 0),) * 2, "off", "raw", "bf16", False),
    # general higher-order rate (last field)
    ("duct_field_f32_omega_hi", (37, 12, 10), 1.0, 0.25, ("periodic", "bounceback", "bounceback"), None, "local",
     "central", "f32", True, 1.6),
    ("periodic_f16_raw_omega_hi", (70, 9, 6), 0.5, 0.25, ("periodic",) * 3, None, "lowmach", "raw", "f16", False, 0.7),
    # stochastic rounding: both layouts key each step's rounding by the same step counter
    ("periodic_bf16_sr_field", (70, 9, 6), 0.5, 0.25, ("periodic",) * 3, None, "local", "central", "bf16_sr", True),
    ("duct_bf16_sr", (37, 12, 10), 1.0, 0.25, ("periodic", "bounceback", "bounceback"), None, "local",
     "central", "bf16_sr", False),
    # nx a multiple of 128: the odd step of two nodes per thread stores whole words across lanes
    ("periodic_f16_words_field", (256, 5, 4), 1.0, 0.5, ("periodic",) * 3, None, "local", "central", "f16", True),
    ("periodic_bf16_sr_words", (128, 6, 5), 0.5, 0.25, ("periodic",) * 3, None, "lowmach", "raw", "bf16_sr", False),
    ("periodic_bf16_words", (384, 3, 4), 1.0, 0.5, ("periodic",) * 3, None, "local", "central", "bf16", True),
]


@pytest.mark.parametrize("case", CASES, ids=[c[0] for c in CASES])
def test_aa_layout_equals_ab_bit_for_bit(case):
    name, (nx, ny, nz), r, s, (bx, by, bz), wv, corr, moments, storage, field = case[:10]
    omega_hi = case[10] if len(case) > 10 else 1.0
    _say("case", name)
    p = oracle.Params(nx, ny, nz, r=r, s=s, omega_nu=1.45, omega_xi=1.2, omega_hi=omega_hi, corr=corr, bc_x=bx,
                      bc_y=by, bc_z=bz, wall_velocity=wv or ((0, 0, 0),) * 6, moments=moments)
    f0 = fp32_rounded_state(random_state(p, 23), p)
    g = np.random.Generator(np.random.PCG64(24))
    force = torch.tensor(1e-4 * g.standard_normal((3, *p.shape))).to(torch.float32).cuda() if field else None
    ab, aa = _lattices(p, storage, force=(1e-5, 0.0, -2e-6))
    a, b = ab.new_state(), ab.new_state()
    ab.import_populations(a, f0.cuda())
    s1 = aa.new_state()
    aa.import_populations(s1, f0.cuda())
    assert torch.equal(ab.export_populations(a), aa.export_populations(s1))
    done = 0
    for n in (2, 4, 10):
        a, b = ab.step(a, b, n, force)
        s1, _ = aa.step(s1, None, n, force)
        done += n
        fa, fb = ab.export_populations(a), aa.export_populations(s1)
        diff = (fa - fb).abs().max().item()
        _say(f"{name}: after {done} steps max |AB - AA| = {diff:.3e}")
        assert torch.equal(fa, fb)
    ma, mb = ab.moments(a, force), aa.moments(s1, force)
    assert torch.equal(ma.rho, mb.rho) and torch.equal(ma.u, mb.u)
    assert torch.equal(ab.density(a), aa.density(s1))


def test_aa_time_dependent_forcing_equals_ab():
    p = oracle.Params(16, 12, 8, r=0.5, s=1.0, omega_nu=1.2, omega_xi=1.2, bc_y="bounceback", bc_z="bounceback")
    forces = np.zeros((40, 3))
    forces[:, 0] = 1e-5 * np.cos(0.05 * np.arange(40))
    ab, aa = _lattices(p, "f32")
    a, b = ab.new_state(), ab.new_state()
    ab.init(a)
    s1 = aa.new_state()
    aa.init(s1)
    a, b = ab.step_forcing(a, b, forces)
    s1, _ = aa.step_forcing(s1, None, forces)
    assert torch.equal(ab.export_populations(a), aa.export_populations(s1))
