"""Seeded synthetic workloads for the cuboid D3Q27 collide-and-stream step.

This module serves both the HIP path's tests/benchmarks and the FP64 oracle.
It holds only input generation -- grids, physical parameters, velocity and
force fields, perturbations -- and none of the method's arithmetic (no
equilibria, moments, relaxation rates or streaming).  Everything is FP64,
NumPy PCG64 with fixed seeds.

Fields are laid out (component, nz, ny, nx); node (i, j, k) sits at the
physical position (i, j r, k s) in lattice units (dx = dt = 1, dy = r, dz = s).
"""

from dataclasses import dataclass, field
import math

import numpy as np

DEFAULT_SEED = 20210730


@dataclass(frozen=True)
class Workload:
    name: str
    nx: int
    ny: int
    nz: int
    r: float
    s: float
    cs2: float
    nu: float
    xi: float
    bc_y: str = "periodic"
    bc_z: str = "periodic"
    steps: int = 0
    storage: str = "f32"
    extra: dict = field(default_factory=dict)

    @property
    def n(self):
        return self.nx * self.ny * self.nz

    @property
    def shape(self):
        return (self.nz, self.ny, self.nx)

    @property
    def extents(self):
        return (self.nx * 1.0, self.ny * self.r, self.nz * self.s)


def _tg_nu(u0, nx, re):
    return u0 * nx / re


def _duct_nu(u_c, ly, lz, re):
    d_h = 2.0 * ly * lz / (ly + lz)
    return u_c * d_h / re


def _tau_nu(tau, cs2):
    return cs2 * (tau - 0.5)


# The five workload definitions.  Readings of under-specified items are listed
# in the design notes (grid aspect ratio = numeric value as the paper's s;
# cs2 = min(r^2, s^2)/3; bulk viscosity equal to shear viscosity; Re on the
# x-extent for the Taylor-Green cases and on the hydraulic diameter for the duct).
TAYLOR_GREEN_32 = Workload(
    "taylor_green_32x32x16", 32, 32, 16, 1.0, 0.5, 1.0 / 12.0,
    nu=_tg_nu(0.05, 32, 100.0), xi=_tg_nu(0.05, 32, 100.0), steps=200,
    extra={"u0": 0.05, "re": 100.0, "noise": 1e-6, "noise_seed": 1})

DUCT_64 = Workload(
    "duct_64x128x32", 64, 128, 32, 1.0, 0.25, 1.0 / 48.0,
    nu=_duct_nu(0.05 * math.sqrt(1.0 / 48.0), 128.0, 8.0, 50.0),
    xi=_duct_nu(0.05 * math.sqrt(1.0 / 48.0), 128.0, 8.0, 50.0),
    bc_y="bounceback", bc_z="bounceback", steps=20000,
    extra={"u_centre": 0.05 * math.sqrt(1.0 / 48.0), "re": 50.0})

DECAYING_512 = Workload(
    "decaying_tg_modes_512x512x256", 512, 512, 256, 1.0, 0.5, 1.0 / 12.0,
    nu=_tg_nu(0.05, 512, 1600.0), xi=_tg_nu(0.05, 512, 1600.0), steps=1000,
    extra={"u0": 0.05, "re": 1600.0, "kmax": 8, "rms": 0.01, "seed": 3})

ADJOINT_DUCT_128 = Workload(
    "adjoint_duct_128x128x64", 128, 128, 64, 1.0, 0.5, 1.0 / 12.0,
    nu=_tau_nu(0.8, 1.0 / 12.0), xi=_tau_nu(0.8, 1.0 / 12.0),
    bc_y="bounceback", bc_z="bounceback", steps=500,
    extra={"force_std": 1e-7, "force_seed": 4, "target_rms": 1e-4, "target_seed": 40,
           "fd_seed": 41, "fd_entries": 16, "checkpoint": 50})

ADJOINT_F16_384 = Workload(
    "adjoint_f16_384x384x192", 384, 384, 192, 0.5, 0.25, 1.0 / 48.0,
    nu=_tau_nu(0.8, 1.0 / 48.0), xi=_tau_nu(0.8, 1.0 / 48.0), steps=1000, storage="f16",
    extra={"kmax": 6, "rms": 0.02, "seed": 5, "target_rms": 0.02, "target_seed": 50,
           "checkpoint": 100})

ALL = (TAYLOR_GREEN_32, DUCT_64, DECAYING_512, ADJOINT_DUCT_128, ADJOINT_F16_384)


def replica(w: Workload, nx, ny, nz, steps=None, name=None):
    """Same physics (r, s, cs2, nu, xi, boundaries) on a smaller grid."""
    return Workload(name or (w.name + f"_replica_{nx}x{ny}x{nz}"), nx, ny, nz, w.r, w.s, w.cs2,
                    w.nu, w.xi, w.bc_y, w.bc_z, w.steps if steps is None else steps,
                    w.storage, dict(w.extra))


# ----------------------------------------------------------------- fields

def coordinates(nx, ny, nz, r, s):
    """Physical node coordinates X, Y, Z, each (nz, ny, nx)."""
    z, y, x = np.meshgrid(np.arange(nz) * s, np.arange(ny) * r, np.arange(nx) * 1.0, indexing="ij")
    return x, y, z


def taylor_green(nx, ny, nz, r, s, u0):
    """u_x = u0 sin(kx x) cos(ky y) cos(kz z), u_y = -u0 (kx/ky) cos sin cos, u_z = 0."""
    x, y, z = coordinates(nx, ny, nz, r, s)
    kx, ky, kz = 2 * math.pi / nx, 2 * math.pi / (ny * r), 2 * math.pi / (nz * s)
    ux = u0 * np.sin(kx * x) * np.cos(ky * y) * np.cos(kz * z)
    uy = -u0 * (kx / ky) * np.cos(kx * x) * np.sin(ky * y) * np.cos(kz * z)
    return np.stack([ux, uy, np.zeros_like(ux)])


def random_modes(nx, ny, nz, r, s, kmax, rms, seed):
    """Solenoidal random field of integer wave indices 1 <= |n| <= kmax.

    Complex Gaussian coefficients (PCG64, ``seed``) on the retained modes,
    projected onto the divergence-free subspace with the physical wave vector
    k_i = 2 pi n_i / L_i, transformed to a real field and scaled so that the
    root-mean-square over all nodes and the three components equals ``rms``.
    """
    rng = np.random.Generator(np.random.PCG64(seed))
    fz = np.fft.fftfreq(nz, 1.0 / nz)
    fy = np.fft.fftfreq(ny, 1.0 / ny)
    fx = np.arange(nx // 2 + 1, dtype=np.float64)
    NZ, NY, NX = np.meshgrid(fz, fy, fx, indexing="ij")
    nmag = np.sqrt(NX ** 2 + NY ** 2 + NZ ** 2)
    mask = (nmag >= 1.0) & (nmag <= kmax)
    idx = np.nonzero(mask)
    m = idx[0].size
    coef = rng.standard_normal((3, m)) + 1j * rng.standard_normal((3, m))
    kvec = np.stack([2 * math.pi * NX[idx] / nx, 2 * math.pi * NY[idx] / (ny * r),
                     2 * math.pi * NZ[idx] / (nz * s)])
    kk = (kvec * kvec).sum(0)
    coef = coef - kvec * ((kvec * coef).sum(0) / kk)
    out = np.empty((3, nz, ny, nx))
    for c in range(3):
        spec = np.zeros((nz, ny, nx // 2 + 1), dtype=np.complex128)
        spec[idx] = coef[c]
        out[c] = np.fft.irfftn(spec, s=(nz, ny, nx), axes=(0, 1, 2))
    cur = math.sqrt(float((out * out).mean()))
    return out * (rms / cur) if cur > 0 else out


def wall_envelope(nx, ny, nz, walls_y, walls_z):
    """sin envelope vanishing half a cell outside the first/last node along walled axes."""
    env = np.ones((nz, ny, nx))
    if walls_y:
        env = env * np.sin(math.pi * (np.arange(ny) + 0.5) / ny)[None, :, None]
    if walls_z:
        env = env * np.sin(math.pi * (np.arange(nz) + 0.5) / nz)[:, None, None]
    return env


def uniform_noise(shape, amplitude, seed):
    """i.i.d. uniform values in [-amplitude, amplitude)."""
    rng = np.random.Generator(np.random.PCG64(seed))
    return rng.uniform(-amplitude, amplitude, size=shape)


def gaussian_field(shape, std, seed):
    rng = np.random.Generator(np.random.PCG64(seed))
    return rng.standard_normal(shape) * std


def sample_indices(count, upper, seed):
    """``count`` distinct integers in [0, upper)."""
    rng = np.random.Generator(np.random.PCG64(seed))
    return np.sort(rng.choice(upper, size=count, replace=False))


# ----------------------------------------------------------------- initial fields per workload

def initial_velocity(w: Workload):
    """Initial velocity field (3, nz, ny, nx) of a workload, FP64."""
    e = w.extra
    if w.name.startswith("taylor_green"):
        return taylor_green(w.nx, w.ny, w.nz, w.r, w.s, e["u0"])
    if w.name.startswith("decaying"):
        return (taylor_green(w.nx, w.ny, w.nz, w.r, w.s, e["u0"])
                + random_modes(w.nx, w.ny, w.nz, w.r, w.s, e["kmax"], e["rms"], e["seed"]))
    if w.name.startswith("adjoint_f16"):
        return random_modes(w.nx, w.ny, w.nz, w.r, w.s, e["kmax"], e["rms"], e["seed"])
    return np.zeros((3, w.nz, w.ny, w.nx))


def initial_density(w: Workload):
    return np.ones((w.nz, w.ny, w.nx))


def target_velocity(w: Workload):
    """Target field u* of the adjoint losses (seeded solenoidal modes, wall envelope)."""
    e = w.extra
    kmax = e.get("kmax", 4)
    u = random_modes(w.nx, w.ny, w.nz, w.r, w.s, kmax, 1.0, e["target_seed"])
    u = u * wall_envelope(w.nx, w.ny, w.nz, w.bc_y == "bounceback", w.bc_z == "bounceback")[None]
    cur = math.sqrt(float((u * u).mean()))
    return u * (e["target_rms"] / cur)


def body_force_field(w: Workload):
    """Per-node body force (3, nz, ny, nx) ~ N(0, force_std^2)."""
    return gaussian_field((3, w.nz, w.ny, w.nx), w.extra["force_std"], w.extra["force_seed"])
