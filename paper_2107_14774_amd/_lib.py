"""ctypes binding of ``liblbm.so`` (the C ABI of include/lbm.h).

Argument marshalling only: every function here forwards to the C entry point
of the same name.  Loading fails loudly when the library has not been built.
"""

import ctypes
import os
import re

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "liblbm.so")
HEADER = os.path.join(os.path.dirname(HERE), "include", "lbm.h")

LBM_OK, LBM_EINVAL, LBM_EHIP, LBM_ESTATE, LBM_ENONFINITE = 0, -1, -2, -3, -4
BC = {"periodic": 0, "bounceback": 1}
STORAGE = {"f32": 0, "f16": 1, "bf16": 2, "bf16_sr": 3}
CORR = {"off": 0, "lowmach": 1, "local": 2, "full": 3}
GRAD_MODE = {"exact": 0, "lagged": 1, "exact_drho": 2}
MOMENTS = {"central": 0, "raw": 1}
LAYOUT = {"ab": 0, "aa": 1}


class LbmParams(ctypes.Structure):
    _fields_ = [
        ("nx", ctypes.c_int32), ("ny", ctypes.c_int32), ("nz", ctypes.c_int32),
        ("r", ctypes.c_double), ("s", ctypes.c_double), ("cs2", ctypes.c_double),
        ("omega_nu", ctypes.c_double), ("omega_xi", ctypes.c_double), ("omega_hi", ctypes.c_double),
        ("bc_x", ctypes.c_int32), ("bc_y", ctypes.c_int32), ("bc_z", ctypes.c_int32),
        ("storage", ctypes.c_int32), ("corr", ctypes.c_int32), ("moments", ctypes.c_int32),
        ("layout", ctypes.c_int32),
        ("rho0", ctypes.c_double), ("force", ctypes.c_double * 3),
        ("wall_velocity", (ctypes.c_double * 3) * 6),
    ]


class LbmError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__(f"lbm status {code}: {msg}")
        self.code = code


_lib = None

_P = ctypes.c_void_p
_SIGNATURES = {
    "lbm_relaxation_rates": (ctypes.c_int, [ctypes.c_double, ctypes.c_double, ctypes.c_double,
                                            ctypes.POINTER(ctypes.c_double), ctypes.POINTER(ctypes.c_double)]),
    "lbm_create": (ctypes.c_int, [ctypes.POINTER(LbmParams), ctypes.POINTER(_P)]),
    "lbm_destroy": (None, [_P]),
    "lbm_state_bytes": (ctypes.c_size_t, [_P]),
    "lbm_state_stride": (ctypes.c_int64, [_P]),
    "lbm_num_nodes": (ctypes.c_int64, [_P]),
    "lbm_set_step_counter": (ctypes.c_int, [_P, ctypes.c_uint64]),
    "lbm_step_counter": (ctypes.c_uint64, [_P]),
    "lbm_last_error": (ctypes.c_char_p, []),
    "lbm_init": (ctypes.c_int, [_P, _P, _P, _P, _P, _P]),
    "lbm_import": (ctypes.c_int, [_P, _P, _P, _P]),
    "lbm_export": (ctypes.c_int, [_P, _P, _P, _P]),
    "lbm_export_nodes": (ctypes.c_int, [_P, _P, _P, ctypes.c_int64, _P, _P]),
    "lbm_step": (ctypes.c_int, [_P, ctypes.c_int32, _P, _P, _P, _P]),
    "lbm_density": (ctypes.c_int, [_P, _P, _P, _P]),
    "lbm_set_force": (ctypes.c_int, [_P, ctypes.POINTER(ctypes.c_double)]),
    "lbm_step_forcing": (ctypes.c_int, [_P, ctypes.c_int32, _P, _P, ctypes.POINTER(ctypes.c_double), _P]),
    "lbm_step_full": (ctypes.c_int, [_P, ctypes.c_int32, _P, _P, _P, _P, _P, ctypes.c_int32, _P]),
    "lbm_stream": (ctypes.c_int, [_P, ctypes.c_int32, _P, _P, _P]),
    "lbm_copy": (ctypes.c_int, [_P, _P, ctypes.c_size_t, _P]),
    "lbm_moments": (ctypes.c_int, [_P, _P, _P, _P, _P, _P, _P]),
    "lbm_check_sums": (ctypes.c_int, [_P, _P, _P]),
    "lbm_step_adjoint": (ctypes.c_int, [_P, _P, _P, _P, _P, _P, _P, _P]),
    "lbm_step_adjoint_full": (ctypes.c_int, [_P, ctypes.c_int32, _P, _P, _P, _P, _P, _P, _P, _P, _P, _P]),
    "lbm_step_adjoint_full_noalloc": (ctypes.c_int, [_P, _P, _P, _P, _P, _P, _P, _P]),
    "lbm_density_adjoint": (ctypes.c_int, [_P, _P, _P, _P]),
    "lbm_adjoint_stream": (ctypes.c_int, [_P, _P, _P, _P, _P, _P, _P]),
    "lbm_moments_adjoint": (ctypes.c_int, [_P, _P, _P, _P, _P, _P, _P, _P]),
    "lbm_init_adjoint": (ctypes.c_int, [_P, _P, _P, _P, _P, _P, _P]),
    "lbm_adjoint_to_natural": (ctypes.c_int, [_P, _P, _P, _P]),
    "lbm_adjoint_from_natural": (ctypes.c_int, [_P, _P, _P, _P]),
}


def header_functions():
    """Names of the functions declared in include/lbm.h."""
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(lbm_\w+)\s*\(", text)))


def load():
    """Load liblbm.so once; raise if it is missing (there is no fallback)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise ImportError(f"{LIB_PATH} not built: run `python -m paper_2107_14774_amd.build`")
    lib = ctypes.CDLL(LIB_PATH)
    for name, (res, args) in _SIGNATURES.items():
        fn = getattr(lib, name)
        fn.restype = res
        fn.argtypes = args
    _lib = lib
    return lib


def check(code):
    if code != LBM_OK:
        msg = load().lbm_last_error()
        raise LbmError(code, msg.decode() if msg else "")
    return code


def ptr(t):
    """Device pointer of a tensor (or None -> NULL)."""
    if t is None:
        return None
    return ctypes.c_void_p(t.data_ptr())


def stream_ptr(stream=None):
    import torch
    s = stream if stream is not None else torch.cuda.current_stream()
    return ctypes.c_void_p(s.cuda_stream)
