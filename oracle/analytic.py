"""Closed forms used to pin the oracle (test infrastructure only).

* eq. 53 (and its restatement at the end of App. D): shear viscosity
  nu = cs2 (1/omega_nu - 1/2), bulk viscosity xi = (2 cs2 / 3)(1/omega_xi - 1/2).
* Linear viscous decay rates of the Navier-Stokes equations recovered in
  eq. 51 (with lattice units dt = 1):
    shear wave u_a(x_b)                    : nu k^2
    planar Taylor-Green in the (a, b) plane: nu (k_a^2 + k_b^2)
    standing sound wave along a            : amplitude rate (2 nu / 3 + xi / 2) k^2,
                                             angular frequency cs k.
* Fully developed flow in a rectangular duct |y| <= a, |z| <= b under a
  uniform body force F_x: the Fourier series that generalises eq. 70 (the
  square-duct case a = b = L/2); it solves nu (u_yy + u_zz) = -F_x / rho with
  u = 0 on the four walls.
* Pulsatile flow in that duct under F_x = F_m cos(omega t) (Sec. 5.2): the
  periodic state u = Re[U(y, z) exp(i omega t)] with i omega U = nu lap U + F_m/rho,
  U = 0 on the walls.  Two independent forms: the double eigenfunction series
  (any a, b) and, for the square duct, the single series of Sec. 5.2 with its
  printed garbles repaired (p_n in place of p^n, and the prefactor F_m/(i omega rho)
  that puts the force cos(omega t) in phase; Wo = a sqrt(omega/nu)).
"""

import math

import numpy as np


def omega_from_nu(nu, cs2):
    return 1.0 / (nu / cs2 + 0.5)


def omega_from_xi(xi, cs2):
    return 1.0 / (1.5 * xi / cs2 + 0.5)


def nu_from_omega(omega, cs2):
    return cs2 * (1.0 / omega - 0.5)


def xi_from_omega(omega, cs2):
    return 2.0 * cs2 / 3.0 * (1.0 / omega - 0.5)


def shear_decay_rate(nu, k):
    return nu * k * k


def taylor_green_decay_rate(nu, ka, kb):
    return nu * (ka * ka + kb * kb)


def sound_decay_rate(nu, xi, k):
    return (2.0 * nu / 3.0 + 0.5 * xi) * k * k


def duct_series(y, z, a, b, force_x, rho, nu, nterms=201):
    """u_x(y, z) in the duct |y| <= a, |z| <= b (y, z numpy arrays, broadcast)."""
    y = np.asarray(y, dtype=np.float64)
    z = np.asarray(z, dtype=np.float64)
    pref = 16.0 * a * a * force_x / (math.pi ** 3 * rho * nu)
    out = np.zeros(np.broadcast(y, z).shape)
    for n in range(1, 2 * nterms, 2):
        k = n * math.pi / (2.0 * a)
        sign = -1.0 if ((n - 1) // 2) % 2 else 1.0
        # cosh(k z) / cosh(k b) written with exponentials that cannot overflow
        ratio = (np.exp(k * (np.abs(z) - b)) + np.exp(-k * (np.abs(z) + b))) / (1.0 + math.exp(-2 * k * b))
        out += sign * (1.0 - ratio) * np.cos(k * y) / n ** 3
    return pref * out


def duct_force_for_centre_velocity(u_centre, a, b, rho, nu, nterms=201):
    """F_x that makes the series velocity at the duct centre equal ``u_centre``."""
    return u_centre / duct_series(0.0, 0.0, a, b, 1.0, rho, nu, nterms)


def pulsatile_duct_double_series(y, z, t, a, b, force_amp, omega, rho, nu, nterms=400):
    """u_x(y, z, t) of the periodic state: U = sum over odd m, n of
    (F/rho) c_mn cos(m pi y / 2a) cos(n pi z / 2b) / (i omega + nu lambda_mn),
    c_mn = 16 (-1)^((m-1)/2 + (n-1)/2) / (pi^2 m n), lambda_mn = (m pi/2a)^2 + (n pi/2b)^2."""
    y = np.asarray(y, dtype=np.float64)
    z = np.asarray(z, dtype=np.float64)
    odd = np.arange(1, 2 * nterms, 2, dtype=np.float64)
    km = odd * math.pi / (2.0 * a)
    kn = odd * math.pi / (2.0 * b)
    sign = np.where(((odd - 1) // 2) % 2 == 1, -1.0, 1.0)
    cy = np.cos(np.multiply.outer(y, km)) * (sign / odd)          # (..., M)
    cz = np.cos(np.multiply.outer(z, kn)) * (sign / odd)          # (..., N)
    lam = km[:, None] ** 2 + kn[None, :] ** 2
    coef = (16.0 / math.pi ** 2) * (force_amp / rho) / (1j * omega + nu * lam)
    U = np.einsum("...m,mn,...n->...", cy, coef, cz)
    return np.real(U * np.exp(1j * omega * t))


def pulsatile_square_duct_series(y, z, t, a, force_amp, omega, rho, nu, nterms=400):
    """The single series of Sec. 5.2 for the square duct |y|, |z| <= a (garbles repaired):
    U = F/(i omega rho) (1 - 2 sum_n (-1)^n / p_n [cosh(g_n y/a) cos(p_n z/a)
        + cosh(g_n z/a) cos(p_n y/a)] / cosh(g_n)),  p_n = (2n+1) pi / 2,
    g_n = sqrt(p_n^2 + i Wo^2)."""
    y = np.asarray(y, dtype=np.float64)
    z = np.asarray(z, dtype=np.float64)
    wo2 = a * a * omega / nu
    psi = np.zeros(np.broadcast(y, z).shape, dtype=np.complex128)
    for n in range(nterms):
        pn = (2 * n + 1) * math.pi / 2.0
        g = np.sqrt(pn * pn + 1j * wo2)
        # cosh(g q/a) / cosh(g) without overflow, |q| <= a
        def ratio(q):
            qa = np.abs(q) / a
            return (np.exp(g * (qa - 1.0)) + np.exp(-g * (qa + 1.0))) / (1.0 + np.exp(-2.0 * g))
        psi += ((-1.0) ** n / pn) * (ratio(y) * np.cos(pn * z / a) + ratio(z) * np.cos(pn * y / a))
    U = force_amp / (1j * omega * rho) * (1.0 - 2.0 * psi)
    return np.real(U * np.exp(1j * omega * t))
