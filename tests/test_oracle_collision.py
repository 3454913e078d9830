"""Pins of the oracle's equilibria and collision (single node, no streaming).

Each test compares the oracle with something it does not compute itself:
eq. 10 typed out, the product form of the equilibrium, the textbook cubic
D3Q27 weights, BGK as the special case of equal rates, exact conservation,
the independent central-moment route (eq. 3a + dense solve), the closed-form
strain-rate solution of eq. 65, and the first-order source identity of App. D.
"""

import math

import pytest
import torch

import oracle
from oracle import collision as C
from oracle import direct as D
from oracle import equilibrium as EQ
from oracle import lattice as L

DT = torch.float64


def _rand_state(n, seed, r, s, cs2, amp_u=0.08, noise=2e-3):
    g = torch.Generator().manual_seed(seed)
    rho = 1.0 + 0.05 * (torch.rand(n, generator=g, dtype=DT) - 0.5)
    u = amp_u * (torch.rand(n, 3, generator=g, dtype=DT) - 0.5)
    f = EQ.feq(rho, u, r, s, cs2)
    f = f + noise * (torch.rand(n, 27, generator=g, dtype=DT) - 0.5) * f
    return f, g


# ------------------------------------------------------------------ equilibria

@pytest.mark.parametrize("r,s,cs2", [(1.0, 1.0, 1 / 3), (1.0, 0.5, 1 / 12), (0.5, 0.25, 1 / 48)])
def test_raw_equilibrium_is_eq10(r, s, cs2):
    g = torch.Generator().manual_seed(1)
    rho = 1 + 0.1 * torch.rand(16, generator=g, dtype=DT)
    u = 0.2 * (torch.rand(16, 3, generator=g, dtype=DT) - 0.5)
    m = EQ.raw_equilibrium(rho, u, cs2)
    x, y, z = u[:, 0], u[:, 1], u[:, 2]
    c = cs2
    want = {
        (0, 0, 0): rho, (1, 0, 0): rho * x, (0, 1, 0): rho * y, (0, 0, 1): rho * z,
        (1, 1, 0): rho * x * y, (1, 0, 1): rho * x * z, (0, 1, 1): rho * y * z,
        (2, 0, 0): c * rho + rho * x * x, (0, 2, 0): c * rho + rho * y * y, (0, 0, 2): c * rho + rho * z * z,
        (1, 2, 0): c * rho * x + rho * x * y * y, (1, 0, 2): c * rho * x + rho * x * z * z,
        (2, 1, 0): c * rho * y + rho * x * x * y, (0, 1, 2): c * rho * y + rho * y * z * z,
        (2, 0, 1): c * rho * z + rho * x * x * z, (0, 2, 1): c * rho * z + rho * y * y * z,
        (1, 1, 1): rho * x * y * z,
        (2, 2, 0): c * c * rho + rho * c * (x * x + y * y) + rho * x * x * y * y,
        (2, 0, 2): c * c * rho + rho * c * (x * x + z * z) + rho * x * x * z * z,
        (0, 2, 2): c * c * rho + rho * c * (y * y + z * z) + rho * y * y * z * z,
        (2, 1, 1): rho * (c + x * x) * y * z, (1, 2, 1): rho * (c + y * y) * x * z,
        (1, 1, 2): rho * (c + z * z) * x * y,
        (1, 2, 2): c * c * rho * x + rho * c * x * (y * y + z * z) + rho * x * y * y * z * z,
        (2, 1, 2): c * c * rho * y + rho * c * y * (x * x + z * z) + rho * x * x * y * z * z,
        (2, 2, 1): c * c * rho * z + rho * c * z * (x * x + y * y) + rho * x * x * y * y * z,
        (2, 2, 2): c ** 3 * rho + rho * c * c * (x * x + y * y + z * z)
        + rho * c * (x * x * y * y + y * y * z * z + x * x * z * z) + rho * x * x * y * y * z * z,
    }
    for mnp, val in want.items():
        assert torch.allclose(m[:, L.MIDX[mnp]], val, atol=1e-15, rtol=1e-13), mnp


@pytest.mark.parametrize("r,s,cs2", [(1.0, 0.5, 1 / 12), (0.5, 0.25, 1 / 48), (0.8, 1.3, 0.2)])
def test_feq_product_form(r, s, cs2):
    """f_eq = rho W_x(ebar_x) W_y(ebar_y) W_z(ebar_z), W(0) = 1-(cs2+u^2)/c^2, W(+-) = ((cs2+u^2)/c^2 +- u/c)/2."""
    g = torch.Generator().manual_seed(2)
    rho = 1 + 0.1 * torch.rand(10, generator=g, dtype=DT)
    u = 0.2 * (torch.rand(10, 3, generator=g, dtype=DT) - 0.5)
    f = EQ.feq(rho, u, r, s, cs2)
    speeds = (1.0, r, s)
    eb = L.ebar()
    want = rho[:, None].expand(10, 27).clone()
    for d in range(3):
        c = speeds[d]
        q = (cs2 + u[:, d] ** 2) / c ** 2
        W0 = 1 - q
        Wp = 0.5 * (q + u[:, d] / c)
        Wm = 0.5 * (q - u[:, d] / c)
        for a in range(27):
            want[:, a] *= {0: W0, 1: Wp, -1: Wm}[int(eb[a, d])]
    assert torch.allclose(f, want, atol=1e-15, rtol=1e-13)


def test_cubic_rest_weights():
    w = EQ.rest_weights(1.0, 1.0, 1.0 / 3.0)
    want = {0: 8 / 27, 1: 2 / 27, 2: 1 / 54, 3: 1 / 216}
    eb = L.ebar()
    for a in range(27):
        assert w[a].item() == pytest.approx(want[int(eb[a].abs().sum())], rel=1e-15)


@pytest.mark.parametrize("r,s,cs2", [(1.0, 0.5, 1 / 12), (0.5, 0.25, 1 / 48)])
def test_feq_central_moments(r, s, cs2):
    """Central moments of f_eq (eq. 3a evaluated directly) are those of eq. 9."""
    g = torch.Generator().manual_seed(3)
    rho = 1 + 0.1 * torch.rand(6, generator=g, dtype=DT)
    u = 0.2 * (torch.rand(6, 3, generator=g, dtype=DT) - 0.5)
    f = EQ.feq(rho, u, r, s, cs2)
    k = torch.einsum("nka,na->nk", D.central_moment_matrix(u, r, s), f)
    assert torch.allclose(k, EQ.central_equilibrium(rho, cs2), atol=1e-14)


# ------------------------------------------------------------------ collision special cases

@pytest.mark.parametrize("r,s,cs2", [(1.0, 1.0, 1 / 3), (0.7, 0.4, 0.04)])
def test_all_rates_one_gives_equilibrium(r, s, cs2):
    p = oracle.Params(1, 1, 1, r=r, s=s, cs2=cs2, omega_nu=1.0, omega_xi=1.0, omega_hi=1.0, corr="off")
    f, _ = _rand_state(20, 4, r, s, cs2)
    rho, u = C.macroscopic(f, torch.zeros(20, 3, dtype=DT), p)
    ft = C.collide(f, torch.zeros(20, 3, dtype=DT), p)
    assert torch.allclose(ft, EQ.feq(rho, u, r, s, cs2), atol=1e-15, rtol=1e-13)


@pytest.mark.parametrize("omega", [0.6, 1.3, 1.8])
def test_equal_rates_give_bgk(omega):
    r, s, cs2 = 0.8, 0.6, 0.1
    p = oracle.Params(1, 1, 1, r=r, s=s, cs2=cs2, omega_nu=omega, omega_xi=omega, omega_hi=omega,
                      omega_1=omega, corr="off")
    f, _ = _rand_state(20, 5, r, s, cs2)
    zero = torch.zeros(20, 3, dtype=DT)
    rho, u = C.macroscopic(f, zero, p)
    ft = C.collide(f, zero, p)
    want = (1 - omega) * f + omega * EQ.feq(rho, u, r, s, cs2)
    assert torch.allclose(ft, want, atol=1e-14)


@pytest.mark.parametrize("corr", ["off", "lowmach", "local", "full"])
def test_conservation_and_source(corr):
    r, s, cs2 = 0.5, 0.25, 1 / 48
    p = oracle.Params(1, 1, 1, r=r, s=s, cs2=cs2, omega_nu=1.5, omega_xi=1.2, corr=corr)
    f, g = _rand_state(30, 6, r, s, cs2, amp_u=0.03)
    force = 1e-3 * (torch.rand(30, 3, generator=g, dtype=DT) - 0.5)
    grad = 1e-3 * (torch.rand(30, 3, generator=g, dtype=DT) - 0.5)
    ft = C.collide(f, force, p, grad_rho=grad)
    e = L.velocities(r, s)
    assert torch.allclose(ft.sum(-1), f.sum(-1), atol=1e-15, rtol=1e-14)
    assert torch.allclose(ft @ e, f @ e + force, atol=1e-15)
    # post-collision first-order central moments are F/2 for any omega_1 (App. D)
    rho, u = C.macroscopic(f, force, p)
    k1 = torch.einsum("nka,na->nk", D.central_moment_matrix(u, r, s), ft)[:, 1:4]
    assert torch.allclose(k1, 0.5 * force, atol=1e-15)


@pytest.mark.parametrize("corr", ["off", "lowmach", "local", "full"])
@pytest.mark.parametrize("r,s", [(1.0, 0.5), (0.5, 0.25), (1.4, 0.7)])
def test_factor_chain_equals_direct_route(corr, r, s):
    cs2 = min(r * r, s * s) / 3
    p = oracle.Params(1, 1, 1, r=r, s=s, omega_nu=1.4, omega_xi=1.1, omega_hi=0.9, corr=corr)
    f, g = _rand_state(40, 7, r, s, cs2)
    force = 1e-3 * (torch.rand(40, 3, generator=g, dtype=DT) - 0.5)
    grad = 1e-2 * (torch.rand(40, 3, generator=g, dtype=DT) - 0.5)
    a = C.collide(f, force, p, grad_rho=grad)
    b = D.collide(f, force, p, grad_rho=grad)
    assert torch.allclose(a, b, atol=1e-14)


def test_uniform_equilibrium_is_fixed_point():
    r, s, cs2 = 0.5, 0.25, 1 / 48
    p = oracle.Params(1, 1, 1, r=r, s=s, omega_nu=1.6, omega_xi=1.3, corr="local")
    rho = torch.full((5,), 1.02, dtype=DT)
    u = torch.tensor([[0.01, -0.02, 0.005]] * 5, dtype=DT)
    f = EQ.feq(rho, u, r, s, cs2)
    ft = C.collide(f, torch.zeros(5, 3, dtype=DT), p)
    assert torch.allclose(ft, f, atol=1e-16, rtol=1e-14)


def test_lowmach_cubic_limit_has_no_correction():
    """At r = s = 1, cs2 = 1/3 the low-Mach corrections vanish (remark in Sec. 2.4)."""
    p_low = oracle.Params(1, 1, 1, r=1.0, s=1.0, cs2=1 / 3, omega_nu=1.3, omega_xi=1.1, corr="lowmach")
    p_off = oracle.Params(1, 1, 1, r=1.0, s=1.0, cs2=1 / 3, omega_nu=1.3, omega_xi=1.1, corr="off")
    f, g = _rand_state(25, 8, 1.0, 1.0, 1 / 3)
    force = 1e-3 * (torch.rand(25, 3, generator=g, dtype=DT) - 0.5)
    assert torch.allclose(C.collide(f, force, p_low), C.collide(f, force, p_off), atol=1e-16, rtol=1e-15)
    # with the 3u^2 terms the corrections do not vanish (they are not grid corrections)
    p_loc = oracle.Params(1, 1, 1, r=1.0, s=1.0, cs2=1 / 3, omega_nu=1.3, omega_xi=1.1, corr="local")
    assert (C.collide(f, force, p_loc) - C.collide(f, force, p_off)).abs().max() > 1e-10


def test_strain_rate_closed_form():
    """The dense solve of App. D's 3x3 system equals its closed-form solution (eq. 65)."""
    r, s = 0.5, 0.25
    p = oracle.Params(1, 1, 1, r=r, s=s, omega_nu=1.5, omega_xi=1.2, corr="local")
    f, _ = _rand_state(12, 9, r, s, p.cs2)
    zero = torch.zeros(12, 3, dtype=DT)
    _, info = C.collide(f, zero, p, return_info=True)
    rho, u, mc = info["rho"], info["u"], info["mc"]
    k200, k020, k002 = (mc[:, L.MIDX[m]] for m in ((2, 0, 0), (0, 2, 0), (0, 0, 2)))
    R_b = k200 + k020 + k002 - 3 * p.cs2 * rho
    R_s1, R_s2 = k200 - k020, k200 - k002
    cs2, wn, wx = p.cs2, p.omega_nu, p.omega_xi
    ux, uy, uz = u[:, 0], u[:, 1], u[:, 2]
    C_sx = (-2 * cs2 / wn + (3 * cs2 - 1) / 2 + 1.5 * ux ** 2) * rho
    C_bx = (-2 * cs2 / wx + (3 * cs2 - 1) / 2 + 1.5 * ux ** 2) * rho
    C_sy = (2 * cs2 / wn - (3 * cs2 - r * r) / 2 - 1.5 * uy ** 2) * rho
    C_by = (-2 * cs2 / wx + (3 * cs2 - r * r) / 2 + 1.5 * uy ** 2) * rho
    C_sz = (2 * cs2 / wn - (3 * cs2 - s * s) / 2 - 1.5 * uz ** 2) * rho
    C_bz = (-2 * cs2 / wx + (3 * cs2 - s * s) / 2 + 1.5 * uz ** 2) * rho
    dxux = ((-C_sz * C_by * R_s1 - C_sy * (C_bz * R_s2 - C_sz * R_b))
            / (-C_sx * C_sz * C_by - C_sy * (C_sx * C_bz - C_sz * C_bx)))
    dyuy = (R_s1 - C_sx * dxux) / C_sy
    dzuz = (R_s2 - C_sx * dxux) / C_sz
    assert torch.allclose(info["du"], torch.stack([dxux, dyuy, dzuz], -1), atol=1e-14, rtol=1e-10)


# ------------------------------------------------------------------ density gradient of the full corrections

def _tensor_weights(r, s, cs2):
    """1D weights per axis (ebar = -1, 0, +1) with speed c: side cs2/(2c^2), centre 1 - cs2/c^2."""
    return [(cs2 / (2 * c * c), 1 - cs2 / (c * c), cs2 / (2 * c * c)) for c in (1.0, r, s)]


@pytest.mark.parametrize("r,s", [(1.0, 0.5), (0.5, 0.25), (1.3, 0.8)])
def test_isotropic_density_gradient_fourier_symbol(r, s):
    """On rho = cos(phase) the lattice-weighted stencil has the closed-form symbol
    d_x -> -sin(th_x) T_y T_z sin(phase), d_y -> -sin(th_y)/r T_x T_z sin(phase), ...
    with T_d = 1 - (cs2/c_d^2)(1 - cos th_d), th_d the phase step per node along d."""
    from oracle import lbm as OL
    nx, ny, nz = 9, 7, 6
    p = oracle.Params(nx, ny, nz, r=r, s=s, corr="full")
    z, y, x = torch.meshgrid(torch.arange(nz, dtype=DT), torch.arange(ny, dtype=DT),
                             torch.arange(nx, dtype=DT), indexing="ij")
    for kx, ky, kz, ph in ((1, 2, 1, 0.3), (4, 1, 2, 1.1), (0, 3, 5, -0.7)):
        th = (2 * math.pi * kx / nx, 2 * math.pi * ky / ny, 2 * math.pi * kz / nz)
        phase = th[0] * x + th[1] * y + th[2] * z + ph
        g = OL.density_gradient(torch.cos(phase), p)
        T = [1 - (p.cs2 / c ** 2) * (1 - math.cos(t)) for c, t in zip((1.0, r, s), th)]
        want = [-math.sin(th[0]) * T[1] * T[2] * torch.sin(phase),
                 -math.sin(th[1]) / r * T[0] * T[2] * torch.sin(phase),
                 -math.sin(th[2]) / s * T[0] * T[1] * torch.sin(phase)]
        for d in range(3):
            assert torch.allclose(g[d], want[d], atol=1e-14), (kx, ky, kz, d)


def test_density_gradient_exact_for_quadratics_and_mirrored_at_walls():
    from oracle import lbm as OL
    r, s = 0.5, 0.25
    # (a) second order: exact on a quadratic field away from the walls (interior nodes)
    p = oracle.Params(8, 7, 6, r=r, s=s, corr="full", bc_y="bounceback", bc_z="bounceback")
    z, y, x = torch.meshgrid(torch.arange(6, dtype=DT) * s, torch.arange(7, dtype=DT) * r,
                             torch.arange(8, dtype=DT), indexing="ij")
    # x is periodic, so the x-dependence is a single Fourier mode scaled by its known symbol
    rho = 1 + 0.1 * y - 0.2 * z + 0.05 * y * y + 0.03 * y * z - 0.07 * z * z
    g = OL.density_gradient(rho, p)
    inner = (slice(1, -1), slice(1, -1), slice(None))
    assert torch.allclose(g[0][inner], torch.zeros_like(g[0][inner]), atol=1e-14)
    assert torch.allclose(g[1][inner], (0.1 + 0.1 * y + 0.03 * z)[inner], atol=1e-13)
    assert torch.allclose(g[2][inner], (-0.2 + 0.03 * y - 0.14 * z)[inner], atol=1e-13)
    # (b) walls: the stencil equals the periodic one on the domain doubled by reflection about each wall
    n_y, n_z = 5, 4
    pw = oracle.Params(6, n_y, n_z, r=r, s=s, corr="full", bc_y="bounceback", bc_z="bounceback")
    pp = oracle.Params(6, 2 * n_y, 2 * n_z, r=r, s=s, corr="full")
    g0 = torch.Generator().manual_seed(3)
    base = torch.rand((n_z, n_y, 6), generator=g0, dtype=DT)
    big = torch.cat([base, base.flip(1)], 1)
    big = torch.cat([big, big.flip(0)], 0)
    want = OL.density_gradient(big, pp)[:, :n_z, :n_y]
    assert torch.allclose(OL.density_gradient(base, pw), want, atol=1e-14)


# ------------------------------------------------------------------ raw-moment scheme (Sec. 7)

def _orders(mask_fn):
    return torch.tensor([mask_fn(sum(mn)) for mn in L.MOMENTS])


@pytest.mark.parametrize("corr", ["off", "lowmach", "local", "full"])
@pytest.mark.parametrize("r,s", [(1.0, 0.5), (0.5, 0.25)])
def test_raw_scheme_equals_central_up_to_second_order(corr, r, s):
    """Relaxing raw or central moments gives the same post-collision moments of order <= 2
    (the non-equilibrium second-order parts and the source images agree, Sec. 2.4) and
    different higher-order moments (the central frame carries u x non-equilibrium terms)."""
    cs2 = min(r * r, s * s) / 3
    kw = dict(r=r, s=s, omega_nu=1.45, omega_xi=1.2, corr=corr)
    pc, pr = oracle.Params(1, 1, 1, **kw), oracle.Params(1, 1, 1, moments="raw", **kw)
    f, g = _rand_state(30, 31, r, s, cs2, amp_u=0.04)
    force = 1e-3 * (torch.rand(30, 3, generator=g, dtype=DT) - 0.5)
    grad = 1e-2 * (torch.rand(30, 3, generator=g, dtype=DT) - 0.5)
    Q = L.P_matrix() * L.S_diag(r, s)[:, None]
    mc = C.collide(f, force, pc, grad_rho=grad) @ Q.T
    mr = C.collide(f, force, pr, grad_rho=grad) @ Q.T
    low = _orders(lambda o: o <= 2)
    assert torch.allclose(mc[:, low], mr[:, low], atol=1e-14)
    assert (mc[:, ~low] - mr[:, ~low]).abs().max() > 1e-8


def test_raw_scheme_higher_moments_are_equilibrium_plus_half_source():
    """With unit higher-order rates the raw scheme sets every raw moment of order >= 3 to its
    equilibrium (eq. 10) plus half the raw image of the central source (eq. 11c)."""
    r, s = 0.7, 0.4
    cs2 = min(r * r, s * s) / 3
    p = oracle.Params(1, 1, 1, r=r, s=s, omega_nu=1.3, omega_xi=1.1, corr="local", moments="raw")
    f, g = _rand_state(20, 32, r, s, cs2, amp_u=0.04)
    force = 1e-3 * (torch.rand(20, 3, generator=g, dtype=DT) - 0.5)
    rho, u = C.macroscopic(f, force, p)
    Q = L.P_matrix() * L.S_diag(r, s)[:, None]
    m = C.collide(f, force, p) @ Q.T
    Finv = L.frame_matrix_inverse(u)
    want = torch.einsum("nab,nb->na", Finv, EQ.central_equilibrium(rho, cs2) + 0.5 * EQ.central_source(force))
    hi = _orders(lambda o: o >= 3)
    assert torch.allclose(m[:, hi], want[:, hi], atol=1e-15)


def test_raw_scheme_without_corrections_at_unit_rates_is_the_central_scheme():
    r, s = 0.5, 0.25
    cs2 = min(r * r, s * s) / 3
    kw = dict(r=r, s=s, omega_nu=1.0, omega_xi=1.0, corr="off")
    f, g = _rand_state(20, 33, r, s, cs2)
    force = 1e-3 * (torch.rand(20, 3, generator=g, dtype=DT) - 0.5)
    a = C.collide(f, force, oracle.Params(1, 1, 1, **kw))
    b = C.collide(f, force, oracle.Params(1, 1, 1, moments="raw", **kw))
    assert torch.allclose(a, b, atol=1e-15)
