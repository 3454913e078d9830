"""Python binding of the cuboid D3Q27 central-moment step (arXiv:2107.14774).

The functions ``lbm_create`` ... ``lbm_adjoint_from_natural`` mirror the C
entry points of include/lbm.h one to one and only marshal arguments: PyTorch
tensors supply device memory and the current HIP stream, every step of the
method runs in the HIP kernels of ``liblbm.so``.  ``Lattice`` bundles a
handle with state allocation for convenience.

Tensor conventions (see include/lbm.h): fields are [3, nz, ny, nx] / [nz, ny,
nx] (SoA, x fastest), natural populations [27, nz, ny, nx] float64, states
are opaque uint8 tensors of ``lbm_state_bytes`` bytes, adjoints float32
[27 * stride] in the state's blocked layout, in gathered-population order
(the element of slot (a, x) is the cotangent of what node x gathers as f_a).
"""

from dataclasses import dataclass

import torch

from . import _lib

_ABI_F32 = torch.float32
_ABI_F64 = torch.float64


def lbm_relaxation_rates(nu, xi, cs2):
    """(omega_nu, omega_xi) from shear and bulk viscosity (eq. 53), computed by the library."""
    on, ox = _lib.ctypes.c_double(), _lib.ctypes.c_double()
    _lib.check(_lib.load().lbm_relaxation_rates(float(nu), float(xi), float(cs2), _lib.ctypes.byref(on),
                                                _lib.ctypes.byref(ox)))
    return on.value, ox.value


relaxation_rates = lbm_relaxation_rates


class Handle:
    """Owns an ``lbm_handle*``."""

    def __init__(self, raw, params):
        self.raw = raw
        self.params = params

    def __del__(self):
        raw, self.raw = getattr(self, "raw", None), None
        if raw:
            try:
                _lib.load().lbm_destroy(raw)
            except Exception:  # interpreter shutdown
                pass

    @property
    def n(self):
        return int(_lib.load().lbm_num_nodes(self.raw))

    @property
    def stride(self):
        return int(_lib.load().lbm_state_stride(self.raw))

    @property
    def state_bytes(self):
        return int(_lib.load().lbm_state_bytes(self.raw))

    @property
    def step_counter(self):
        return int(_lib.load().lbm_step_counter(self.raw))


def lbm_set_step_counter(h, counter):
    _lib.check(_lib.load().lbm_set_step_counter(h.raw, int(counter)))


def lbm_step_counter(h):
    return int(_lib.load().lbm_step_counter(h.raw))


def _require(t, dtype, numel, name):
    if t is None:
        return None
    if not t.is_cuda or t.dtype != dtype or not t.is_contiguous() or t.numel() != numel:
        raise ValueError(f"{name}: need a contiguous CUDA {dtype} tensor of {numel} elements, "
                         f"got {t.dtype} {tuple(t.shape)} on {t.device}")
    return t


def _state(h, t, name="state"):
    if t is None or not t.is_cuda or not t.is_contiguous() or t.numel() * t.element_size() < h.state_bytes:
        raise ValueError(f"{name}: need a contiguous CUDA buffer of >= {h.state_bytes} bytes")
    return t


def lbm_create(nx, ny, nz, r=1.0, s=1.0, cs2=0.0, omega_nu=1.0, omega_xi=1.0, omega_hi=1.0,
               bc_y="periodic", bc_z="periodic", storage="f32", corr="local", rho0=1.0,
               force=(0.0, 0.0, 0.0), bc_x="periodic", wall_velocity=None, moments="central", layout="ab"):
    """wall_velocity: None or six 3-vectors, faces x-, x+, y-, y+, z-, z+."""
    lib = _lib.load()
    p = _lib.LbmParams()
    p.nx, p.ny, p.nz = nx, ny, nz
    p.r, p.s, p.cs2 = r, s, cs2
    p.omega_nu, p.omega_xi, p.omega_hi = omega_nu, omega_xi, omega_hi
    p.bc_x, p.bc_y, p.bc_z = _lib.BC[bc_x], _lib.BC[bc_y], _lib.BC[bc_z]
    p.storage, p.corr = _lib.STORAGE[storage], _lib.CORR[corr]
    p.moments = _lib.MOMENTS[moments]
    p.layout = _lib.LAYOUT[layout]
    p.rho0 = rho0
    for d in range(3):
        p.force[d] = float(force[d])
    if wall_velocity is not None:
        if len(wall_velocity) != 6:
            raise ValueError("wall_velocity: six faces (x-, x+, y-, y+, z-, z+)")
        for f, v in enumerate(wall_velocity):
            for d in range(3):
                p.wall_velocity[f][d] = float(v[d])
    raw = _lib.ctypes.c_void_p()
    _lib.check(lib.lbm_create(_lib.ctypes.byref(p), _lib.ctypes.byref(raw)))
    return Handle(raw, p)


def lbm_init(h, state, rho=None, u=None, perturb=None, stream=None):
    n = h.n
    _require(rho, _ABI_F64, n, "rho")
    _require(u, _ABI_F64, 3 * n, "u")
    _require(perturb, _ABI_F64, 27 * n, "perturb")
    _lib.check(_lib.load().lbm_init(h.raw, _lib.ptr(_state(h, state)), _lib.ptr(rho), _lib.ptr(u),
                                    _lib.ptr(perturb), _lib.stream_ptr(stream)))


def lbm_import(h, state, f, stream=None):
    _require(f, _ABI_F64, 27 * h.n, "f")
    _lib.check(_lib.load().lbm_import(h.raw, _lib.ptr(_state(h, state)), _lib.ptr(f), _lib.stream_ptr(stream)))


def lbm_export(h, state, f, stream=None):
    _require(f, _ABI_F64, 27 * h.n, "f")
    _lib.check(_lib.load().lbm_export(h.raw, _lib.ptr(_state(h, state)), _lib.ptr(f), _lib.stream_ptr(stream)))


def lbm_export_nodes(h, state, nodes, f, stream=None):
    """``nodes``: device int64 [count]; ``f``: device float64 [27, count]."""
    count = nodes.numel()
    _require(nodes, torch.int64, count, "nodes")
    _require(f, _ABI_F64, 27 * count, "f")
    _lib.check(_lib.load().lbm_export_nodes(h.raw, _lib.ptr(_state(h, state)), _lib.ptr(nodes), count, _lib.ptr(f),
                                            _lib.stream_ptr(stream)))


def _state_b(h, t):
    """state_b: a buffer, or None in the AA layout (one buffer updated in place)."""
    return None if t is None and h.params.layout == _lib.LAYOUT["aa"] else _state(h, t, "state_b")


def lbm_step(h, nsteps, state_a, state_b, force=None, stream=None):
    _require(force, _ABI_F32, 3 * h.n, "force")
    _lib.check(_lib.load().lbm_step(h.raw, int(nsteps), _lib.ptr(_state(h, state_a)),
                                    _lib.ptr(_state_b(h, state_b)), _lib.ptr(force),
                                    _lib.stream_ptr(stream)))


def lbm_set_force(h, force):
    arr = (_lib.ctypes.c_double * 3)(*(float(v) for v in force))
    _lib.check(_lib.load().lbm_set_force(h.raw, arr))


def lbm_step_forcing(h, nsteps, state_a, state_b, forces, stream=None):
    """``forces``: host sequence or array of nsteps uniform forces (nsteps x 3)."""
    import numpy as np
    arr = np.ascontiguousarray(np.asarray(forces, dtype=np.float64).reshape(-1))
    if arr.size != 3 * int(nsteps):
        raise ValueError(f"forces: need {nsteps} x 3 values, got {arr.size}")
    ptr = arr.ctypes.data_as(_lib.ctypes.POINTER(_lib.ctypes.c_double))
    _lib.check(_lib.load().lbm_step_forcing(h.raw, int(nsteps), _lib.ptr(_state(h, state_a)),
                                            _lib.ptr(_state_b(h, state_b)), ptr,
                                            _lib.stream_ptr(stream)))


def lbm_density(h, state, drho, stream=None):
    _require(drho, _ABI_F32, h.n, "drho")
    _lib.check(_lib.load().lbm_density(h.raw, _lib.ptr(_state(h, state)), _lib.ptr(drho), _lib.stream_ptr(stream)))


def lbm_step_full(h, nsteps, state_a, state_b, drho_a, drho_b=None, mode="lagged", force=None, stream=None):
    """Steps with the full corrections; ``mode`` is "exact" or "lagged" (see include/lbm.h)."""
    _require(force, _ABI_F32, 3 * h.n, "force")
    _require(drho_a, _ABI_F32, h.n, "drho_a")
    _require(drho_b, _ABI_F32, h.n, "drho_b")
    _lib.check(_lib.load().lbm_step_full(h.raw, int(nsteps), _lib.ptr(_state(h, state_a)),
                                         _lib.ptr(_state(h, state_b, "state_b")), _lib.ptr(force),
                                         _lib.ptr(drho_a), _lib.ptr(drho_b), _lib.GRAD_MODE[mode],
                                         _lib.stream_ptr(stream)))


def lbm_stream(h, nsteps, state_a, state_b, stream=None):
    _lib.check(_lib.load().lbm_stream(h.raw, int(nsteps), _lib.ptr(_state(h, state_a)),
                                      _lib.ptr(_state(h, state_b, "state_b")), _lib.stream_ptr(stream)))


def lbm_copy(dst, src, nbytes=None, stream=None):
    """Copy ``nbytes`` (default: all of ``src``) between two device tensors."""
    nbytes = src.numel() * src.element_size() if nbytes is None else int(nbytes)
    for t, name in ((dst, "dst"), (src, "src")):
        if not t.is_cuda or not t.is_contiguous() or t.numel() * t.element_size() < nbytes:
            raise ValueError(f"{name}: need a contiguous device tensor of at least {nbytes} bytes")
    _lib.check(_lib.load().lbm_copy(_lib.ptr(dst), _lib.ptr(src), nbytes, _lib.stream_ptr(stream)))


def lbm_moments(h, state, force=None, rho=None, u=None, sums=None, stream=None):
    n = h.n
    _require(force, _ABI_F32, 3 * n, "force")
    _require(rho, _ABI_F32, n, "rho")
    _require(u, _ABI_F32, 3 * n, "u")
    _require(sums, _ABI_F64, 5, "sums")
    _lib.check(_lib.load().lbm_moments(h.raw, _lib.ptr(_state(h, state)), _lib.ptr(force), _lib.ptr(rho),
                                       _lib.ptr(u), _lib.ptr(sums), _lib.stream_ptr(stream)))


def lbm_check_sums(sums, stream=None):
    """Synchronising NaN/Inf check of the five totals; returns them as a list."""
    _require(sums, _ABI_F64, 5, "sums")
    out = (_lib.ctypes.c_double * 5)()
    _lib.check(_lib.load().lbm_check_sums(_lib.ptr(sums), out, _lib.stream_ptr(stream)))
    return list(out)


def lbm_step_adjoint(h, state_t, adj_in, adj_out, force=None, grad_force=None, grad_force_uniform=None,
                     stream=None):
    m = 27 * h.stride
    _require(adj_in, _ABI_F32, m, "adj_in")
    _require(adj_out, _ABI_F32, m, "adj_out")
    _require(force, _ABI_F32, 3 * h.n, "force")
    _require(grad_force, _ABI_F32, 3 * h.n, "grad_force")
    _require(grad_force_uniform, _ABI_F64, 3, "grad_force_uniform")
    _lib.check(_lib.load().lbm_step_adjoint(h.raw, _lib.ptr(_state(h, state_t)), _lib.ptr(adj_in),
                                            _lib.ptr(adj_out), _lib.ptr(force), _lib.ptr(grad_force),
                                            _lib.ptr(grad_force_uniform), _lib.stream_ptr(stream)))


def lbm_step_adjoint_full(h, state_t, adj_in, adj_out, drho, grad_work, force=None, grad_force=None,
                          grad_force_uniform=None, mode="exact", grad_pending=None, stream=None):
    """Adjoint step of the full corrections; ``mode`` "exact", "exact_drho" (exact level, ``drho``
    already holds the state's density) or "lagged" (see include/lbm.h)."""
    m = 27 * h.stride
    _require(adj_in, _ABI_F32, m, "adj_in")
    _require(adj_out, _ABI_F32, m, "adj_out")
    _require(drho, _ABI_F32, h.n, "drho")
    _require(grad_work, _ABI_F32, 3 * h.n, "grad_work")
    _require(grad_pending, _ABI_F32, 3 * h.n, "grad_pending")
    _require(force, _ABI_F32, 3 * h.n, "force")
    _require(grad_force, _ABI_F32, 3 * h.n, "grad_force")
    _require(grad_force_uniform, _ABI_F64, 3, "grad_force_uniform")
    _lib.check(_lib.load().lbm_step_adjoint_full(h.raw, _lib.GRAD_MODE[mode], _lib.ptr(_state(h, state_t)),
                                                 _lib.ptr(adj_in), _lib.ptr(adj_out), _lib.ptr(force),
                                                 _lib.ptr(grad_force), _lib.ptr(grad_force_uniform), _lib.ptr(drho),
                                                 _lib.ptr(grad_work), _lib.ptr(grad_pending),
                                                 _lib.stream_ptr(stream)))


def lbm_step_adjoint_full_noalloc(h, state_t, adj_in, adj_out, force=None, grad_force=None,
                                  grad_force_uniform=None, stream=None):
    """lbm_step_adjoint_full at the exact time level with the library's static work array (allocates
    nothing; see include/lbm.h)."""
    m = 27 * h.stride
    _require(adj_in, _ABI_F32, m, "adj_in")
    _require(adj_out, _ABI_F32, m, "adj_out")
    _require(force, _ABI_F32, 3 * h.n, "force")
    _require(grad_force, _ABI_F32, 3 * h.n, "grad_force")
    _require(grad_force_uniform, _ABI_F64, 3, "grad_force_uniform")
    _lib.check(_lib.load().lbm_step_adjoint_full_noalloc(h.raw, _lib.ptr(_state(h, state_t)), _lib.ptr(adj_in),
                                                         _lib.ptr(adj_out), _lib.ptr(force), _lib.ptr(grad_force),
                                                         _lib.ptr(grad_force_uniform), _lib.stream_ptr(stream)))


def lbm_adjoint_stream(h, state_t, adj_in, adj_out, force=None, grad_force=None, stream=None):
    """The adjoint step's data movement without its arithmetic (a measured ceiling; see include/lbm.h)."""
    m = 27 * h.stride
    _require(adj_in, _ABI_F32, m, "adj_in")
    _require(adj_out, _ABI_F32, m, "adj_out")
    _require(force, _ABI_F32, 3 * h.n, "force")
    _require(grad_force, _ABI_F32, 3 * h.n, "grad_force")
    _lib.check(_lib.load().lbm_adjoint_stream(h.raw, _lib.ptr(_state(h, state_t)), _lib.ptr(adj_in), _lib.ptr(adj_out),
                                              _lib.ptr(force), _lib.ptr(grad_force), _lib.stream_ptr(stream)))


def lbm_density_adjoint(h, grad, adj, stream=None):
    _require(grad, _ABI_F32, 3 * h.n, "grad")
    _require(adj, _ABI_F32, 27 * h.stride, "adj")
    _lib.check(_lib.load().lbm_density_adjoint(h.raw, _lib.ptr(grad), _lib.ptr(adj), _lib.stream_ptr(stream)))


def lbm_moments_adjoint(h, state, adj, force=None, g_rho=None, g_u=None, grad_force=None, stream=None):
    n = h.n
    _require(adj, _ABI_F32, 27 * h.stride, "adj")
    _require(force, _ABI_F32, 3 * n, "force")
    _require(g_rho, _ABI_F32, n, "g_rho")
    _require(g_u, _ABI_F32, 3 * n, "g_u")
    _require(grad_force, _ABI_F32, 3 * n, "grad_force")
    _lib.check(_lib.load().lbm_moments_adjoint(h.raw, _lib.ptr(_state(h, state)), _lib.ptr(force),
                                               _lib.ptr(g_rho), _lib.ptr(g_u), _lib.ptr(adj),
                                               _lib.ptr(grad_force), _lib.stream_ptr(stream)))


def lbm_init_adjoint(h, adj, rho=None, u=None, g_rho=None, g_u=None, stream=None):
    n = h.n
    _require(adj, _ABI_F32, 27 * h.stride, "adj")
    _require(rho, _ABI_F64, n, "rho")
    _require(u, _ABI_F64, 3 * n, "u")
    _require(g_rho, _ABI_F64, n, "g_rho")
    _require(g_u, _ABI_F64, 3 * n, "g_u")
    _lib.check(_lib.load().lbm_init_adjoint(h.raw, _lib.ptr(adj), _lib.ptr(rho), _lib.ptr(u),
                                            _lib.ptr(g_rho), _lib.ptr(g_u), _lib.stream_ptr(stream)))


def lbm_adjoint_to_natural(h, slots, natural, stream=None):
    _require(slots, _ABI_F32, 27 * h.stride, "slots")
    _require(natural, _ABI_F64, 27 * h.n, "natural")
    _lib.check(_lib.load().lbm_adjoint_to_natural(h.raw, _lib.ptr(slots), _lib.ptr(natural),
                                                  _lib.stream_ptr(stream)))


def lbm_adjoint_from_natural(h, natural, slots, stream=None):
    _require(slots, _ABI_F32, 27 * h.stride, "slots")
    _require(natural, _ABI_F64, 27 * h.n, "natural")
    _lib.check(_lib.load().lbm_adjoint_from_natural(h.raw, _lib.ptr(natural), _lib.ptr(slots),
                                                    _lib.stream_ptr(stream)))


# ---------------------------------------------------------------------- convenience wrapper

@dataclass
class Moments:
    rho: torch.Tensor
    u: torch.Tensor
    sums: torch.Tensor


class Lattice:
    """A handle plus allocation helpers; fields are torch tensors on ``device``."""

    def __init__(self, nx, ny, nz, device="cuda", **kw):
        self.h = lbm_create(nx, ny, nz, **kw)
        self.nx, self.ny, self.nz = nx, ny, nz
        self.shape = (nz, ny, nx)
        self.device = torch.device(device)

    @property
    def n(self):
        return self.h.n

    def new_state(self):
        return torch.empty(self.h.state_bytes, dtype=torch.uint8, device=self.device)

    def new_adjoint(self, zero=True):
        t = torch.empty(27 * self.h.stride, dtype=torch.float32, device=self.device)
        return t.zero_() if zero else t

    def field(self, ncomp, dtype=torch.float32):
        shape = (ncomp, *self.shape) if ncomp > 1 else self.shape
        return torch.empty(shape, dtype=dtype, device=self.device)

    def init(self, state, rho=None, u=None, perturb=None):
        lbm_init(self.h, state, *(None if t is None else t.to(self.device, _ABI_F64).contiguous()
                                  for t in (rho, u, perturb)))
        return state

    def import_populations(self, state, f):
        lbm_import(self.h, state, f.to(self.device, _ABI_F64).contiguous())
        return state

    def export_populations(self, state):
        f = torch.empty((27, *self.shape), dtype=_ABI_F64, device=self.device)
        lbm_export(self.h, state, f)
        return f

    @property
    def aa(self):
        return self.h.params.layout == _lib.LAYOUT["aa"]

    def step(self, a, b, nsteps, force=None):
        """Advance; returns (current, scratch) after nsteps (AA layout: b may be None, a stays current)."""
        lbm_step(self.h, nsteps, a, b, force)
        return (a, b) if (nsteps % 2 == 0 or self.aa) else (b, a)

    def step_full(self, a, b, nsteps, drho_a, drho_b=None, mode="lagged", force=None):
        """Full corrections; returns (current, scratch, current density field, other density field)."""
        lbm_step_full(self.h, nsteps, a, b, drho_a, drho_b, mode, force)
        if nsteps % 2 == 0 or mode == "exact":
            return ((a, b) if nsteps % 2 == 0 else (b, a)) + (drho_a, drho_b)
        return b, a, drho_b, drho_a

    def step_forcing(self, a, b, forces):
        """Advance len(forces) steps, step t under the uniform force forces[t]; returns (current, scratch)."""
        n = len(forces)
        lbm_step_forcing(self.h, n, a, b, forces)
        return (a, b) if (n % 2 == 0 or self.aa) else (b, a)

    def set_force(self, force):
        lbm_set_force(self.h, force)

    def density(self, state):
        """rho - rho0 (FP32 field) of a state."""
        d = self.field(1)
        lbm_density(self.h, state, d)
        return d

    def moments(self, state, force=None, sums=True):
        rho = self.field(1)
        u = self.field(3)
        s = torch.empty(5, dtype=_ABI_F64, device=self.device) if sums else None
        lbm_moments(self.h, state, force, rho, u, s)
        return Moments(rho, u, s)
