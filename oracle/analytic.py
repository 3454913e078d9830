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
