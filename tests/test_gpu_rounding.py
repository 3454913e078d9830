"""GPU checks of the stochastic rounding of BF16-SR storage: the step counter
keys it (same state and counter -> the same bits; another counter -> other
bits, while round-to-nearest BF16 ignores the counter), and it is unbiased
where round-to-nearest is not: a flow whose deviations change by much less
than BF16's resolution per step keeps decaying under stochastic rounding."""

import sys

import pytest
import torch

import oracle
from helpers import gpu_lattice, random_state

pytestmark = pytest.mark.gpu


def _say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


@pytest.mark.parametrize("storage", ["bf16", "bf16_sr"])
def test_step_counter_keys_the_rounding(storage):
    import paper_2107_14774_amd as P
    p = oracle.Params(130, 6, 5, r=1.0, s=0.5, omega_nu=1.4, omega_xi=1.2)
    lat = gpu_lattice(p, storage=storage)
    start = lat.new_state()
    lat.import_populations(start, random_state(p, 91).cuda())
    out = {}
    for counter in (7, 7, 8):
        a, b = lat.new_state(), lat.new_state()
        a.copy_(start)
        P.lbm_set_step_counter(lat.h, counter)
        P.lbm_step(lat.h, 3, a, b)
        assert lat.h.step_counter == counter + 3
        out.setdefault(counter, []).append(lat.export_populations(b))
    same = torch.equal(out[7][0], out[7][1])
    other = torch.equal(out[7][0], out[8][0])
    _say(f"{storage}: same counter reproduces: {same}; another counter gives the same bits: {other}")
    assert same
    assert other == (storage == "bf16")


def test_stochastic_rounding_follows_a_slow_decay():
    """A single shear wave of tiny amplitude decays by about 1e-4 of itself per step, far below BF16's
    relative resolution (2^-9).  Round-to-nearest holds most stored deviations at the same bits; the
    stochastic rounding tracks the FP32 decay in the mean."""
    import numpy as np
    nx, ny, nz = 64, 32, 16
    p = oracle.Params(nx, ny, nz, r=1.0, s=0.5, omega_nu=1.9, omega_xi=1.2)
    y = np.arange(ny) * p.r
    u = np.zeros((3, nz, ny, nx))
    u[0] = 1e-3 * np.sin(2 * np.pi * y / (ny * p.r))[None, :, None]
    u0 = torch.from_numpy(u).cuda()
    amp = {}
    for storage in ("f32", "bf16", "bf16_sr"):
        lat = gpu_lattice(p, storage=storage)
        a, b = lat.new_state(), lat.new_state()
        lat.init(a, u=u0)
        cur, _ = lat.step(a, b, 400)
        m = lat.moments(cur)
        ux = m.u[0].double().mean(dim=(0, 2)).cpu().numpy()          # profile along y
        amp[storage] = float(2 * np.mean(ux * np.sin(2 * np.pi * y / (ny * p.r))))
        _say(f"{storage}: shear-wave amplitude after 400 steps {amp[storage]:.6e}")
    decay = 1e-3 - amp["f32"]
    err_rn, err_sr = abs(amp["bf16"] - amp["f32"]), abs(amp["bf16_sr"] - amp["f32"])
    _say(f"decay {decay:.3e}; |bf16 - f32| {err_rn:.3e}; |bf16_sr - f32| {err_sr:.3e}")
    assert err_sr < 0.25 * decay
    assert err_sr < err_rn
