"""Host-side checks of the example scripts (no GPU): their own closed forms and
search logic against the oracle and against definitions."""

import math

import numpy as np

from oracle import analytic as A
from examples import pulsatile_duct as PD
from examples import shallow_cavity as SC
from examples import stability_sweep as SS


def test_pulsatile_example_series_equals_the_oracle_series():
    a, F, w = 20.0, 1e-5, 2 * math.pi / 10000
    nu = a * a * w / 3.09 ** 2
    g = np.random.default_rng(3)
    y, z = g.uniform(-a, a, 30), g.uniform(-a, a, 30)
    for t in (0.0, 3333.0):
        got = PD.periodic_series(y, z, t, a, F, w, nu)
        want = A.pulsatile_duct_double_series(y, z, t, a, a, F, w, 1.0, nu)
        assert np.abs(got - want).max() < 1e-12 * F / w


def test_bisection_finds_the_threshold():
    runs = []

    def fn(x):
        runs.append(x)
        return x <= 0.2371, 0
    x, n = SS.bisect(fn, 0.0, 0.4, 10)
    assert abs(x - 0.2371) < 0.4 / 2 ** 10 and x <= 0.2371 and n == 11
    assert SS.bisect(lambda x: (True, 0), 0.0, 0.4, 5) == (0.4, 1)


def test_cavity_cases_follow_the_paper_node_counts():
    """Sec. 6: Nx = r (L/H) Ny, Nz = (r/s)(W/H) Ny with L/H = 4, W/H = 2, Ny = 64."""
    for name, c in SC.CASES.items():
        assert c["ny"] == 64
        assert abs(c["nx"] - c["r"] * 4 * 64) < 0.5
        assert abs(c["nz"] - (c["r"] / c["s"]) * 2 * 64) < 0.6, name
    cubic = SC.CASES["cubic"]
    ratios = [cubic["nx"] * cubic["ny"] * cubic["nz"] / (c["nx"] * c["ny"] * c["nz"]) for k, c in SC.CASES.items()
              if k != "cubic"]
    assert [round(q, 2) for q in ratios] == [7.88, 5.33, 7.11]
    assert SC.centre_pair(64) == (31, 32) and SC.centre_pair(41) == (20, 20)
