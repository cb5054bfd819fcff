"""ctypes binding of libibdl.so (argument marshalling only; every step runs in the HIP library)."""
from __future__ import annotations

import ctypes
import os
import re

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libibdl.so")
HEADER = os.path.join(os.path.dirname(_HERE), "include", "ibdl.h")

c_int32, c_int64, c_double, c_void_p = ctypes.c_int32, ctypes.c_int64, ctypes.c_double, ctypes.c_void_p

PDE = {"screened": 0, "poisson": 1, "stokes": 2}
BC = {"dirichlet": 0, "neumann": 1}
KERNEL = {"peskin4": 0, "cos4": 1, "bspline6": 2}
DISC = {"fd2": 0, "spectral": 1}
PRECISION = {"fp64": 0, "mixed": 1}
METHOD = {"dl": 0, "sl": 1}
STATUS = {0: "IBDL_OK", 1: "IBDL_NOT_CONVERGED", -1: "IBDL_ERR_ARG", -2: "IBDL_ERR_UNSUPPORTED",
          -3: "IBDL_ERR_NOMEM", -4: "IBDL_ERR_HIP", -5: "IBDL_ERR_NONFINITE", -6: "IBDL_ERR_STATE"}


class Config(ctypes.Structure):
    _fields_ = [("dim", c_int32), ("n", c_int64 * 3), ("L", c_double * 3), ("origin", c_double * 3),
                ("pde", c_int32), ("kappa", c_double), ("mu", c_double), ("bc", c_int32), ("eta", c_double),
                ("kernel", c_int32), ("disc", c_int32), ("precision", c_int32), ("stream", c_void_p),
                ("method", c_int32)]


class Info(ctypes.Structure):
    _fields_ = [("iters", c_int32), ("status", c_int32), ("krylov_relres", c_double),
                ("true_relres_fp64", c_double), ("history", ctypes.POINTER(c_double)), ("history_cap", c_int32)]


class NSParams(ctypes.Structure):
    _fields_ = [("rho", c_double), ("dt", c_double), ("m1", c_double), ("m2", c_double), ("strip", c_int32),
                ("u_inf", c_double), ("tol", c_double), ("maxit", c_int32)]


_lib = None

_SIGS = {
    "ibdl_create": (c_int32, [ctypes.POINTER(Config), c_int64, c_void_p, c_void_p, c_void_p, ctypes.POINTER(c_void_p)]),
    "ibdl_set_markers": (c_int32, [c_void_p, c_void_p, c_void_p, c_void_p]),
    "ibdl_destroy": (c_int32, [c_void_p]),
    "ibdl_spread": (c_int32, [c_void_p, c_void_p, c_int32, c_void_p]),
    "ibdl_interp": (c_int32, [c_void_p, c_void_p, c_int32, c_void_p]),
    "ibdl_grid_solve": (c_int32, [c_void_p, c_void_p, c_void_p]),
    "ibdl_grid_solve_static": (c_int32, [ctypes.POINTER(Config), c_void_p, c_void_p]),
    "ibdl_apply": (c_int32, [c_void_p, c_void_p, c_void_p]),
    "ibdl_solve": (c_int32, [c_void_p, c_void_p, c_void_p, c_double, c_int32, c_void_p, c_void_p,
                             ctypes.POINTER(Info)]),
    "ibdl_solve_refined": (c_int32, [c_void_p, c_void_p, c_void_p, c_double, c_int32, c_double, c_int32,
                                     c_void_p, c_void_p, ctypes.POINTER(Info)]),
    "ibdl_apply_transpose": (c_int32, [c_void_p, c_void_p, c_void_p]),
    "ibdl_backward": (c_int32, [c_void_p, c_void_p, c_void_p, c_void_p, c_double, c_int32, c_void_p, c_void_p,
                                ctypes.POINTER(Info)]),
    "ibdl_batch_create": (c_int32, [c_int32, c_void_p, c_void_p, c_void_p, c_void_p, c_void_p,
                                    ctypes.POINTER(c_void_p)]),
    "ibdl_batch_destroy": (c_int32, [c_void_p]),
    "ibdl_batch_apply": (c_int32, [c_void_p, c_void_p, c_void_p]),
    "ibdl_batch_solve": (c_int32, [c_void_p, c_void_p, c_double, c_int32, c_void_p, c_void_p, c_void_p]),
    "ibdl_batch_set_graph": (c_int32, [c_void_p, c_int32]),
    "ibdl_batch_query": (c_int32, [c_void_p, c_int32, ctypes.POINTER(c_int32), ctypes.POINTER(c_int32),
                                   ctypes.POINTER(c_int32), ctypes.POINTER(c_int32), ctypes.POINTER(c_int32),
                                   ctypes.POINTER(c_int32)]),
    "ibdl_batch_last_error": (ctypes.c_char_p, [c_void_p]),
    "ibdl_active_rows": (c_int32, [c_void_p, ctypes.POINTER(c_int64), ctypes.POINTER(c_int64)]),
    "ibdl_active_span": (c_int32, [c_void_p, ctypes.POINTER(c_int32), ctypes.POINTER(c_int32)]),
    "ibdl_launch_shape": (c_int32, [c_void_p, ctypes.POINTER(c_int32), ctypes.POINTER(c_int32),
                                    ctypes.POINTER(c_int32)]),
    "ibdl_query": (c_int32, [c_void_p, ctypes.POINTER(c_int64), ctypes.POINTER(c_int64), ctypes.POINTER(c_int32)]),
    "ibdl_last_error": (ctypes.c_char_p, [c_void_p]),
    "ibdl_set_timing": (c_int32, [c_void_p, c_int32]),
    "ibdl_set_graph": (c_int32, [c_void_p, c_int32]),
    "ibdl_spread_tiles": (c_int32, [c_void_p, c_void_p, c_void_p, c_void_p]),
    "ibdl_indicator": (c_int32, [c_void_p, c_void_p, c_void_p]),
    "ibdl_near_boundary": (c_int32, [c_void_p, c_void_p, c_void_p, c_void_p, c_double, c_double, c_void_p]),
    "ibdl_near_widths": (c_int32, [c_void_p, c_void_p, c_void_p]),
    "ibdl_advection": (c_int32, [c_void_p, c_void_p, c_void_p]),
    "ibdl_ns_step": (c_int32, [c_void_p, ctypes.POINTER(NSParams), c_void_p, c_void_p, c_void_p, c_void_p, c_void_p,
                               c_void_p, c_void_p, c_void_p, ctypes.POINTER(Info)]),
    "ibdl_pressure": (c_int32, [c_void_p, c_void_p, c_void_p, c_void_p]),
    "ibdl_cv_force": (c_int32, [c_void_p, c_void_p, c_void_p, c_double, c_void_p, c_void_p, c_double, c_void_p,
                                c_void_p]),
    "ibdl_net_force": (c_int32, [c_void_p, c_void_p, c_void_p]),
    "ibdl_line_integral": (c_int32, [c_void_p, c_void_p, c_int32, c_int32, c_int64, c_void_p]),
    "ibdl_get_timing": (c_int32, [c_void_p, ctypes.POINTER(c_double), ctypes.POINTER(c_int64), c_int32]),
}


def load():
    """Load the in-tree HIP library; raises if it has not been built (there is no fallback)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(f"{LIB_PATH} is missing: build it with `python -m paper_2210_07403_amd.build`")
        lib = ctypes.CDLL(LIB_PATH)
        for name, (res, args) in _SIGS.items():
            fn = getattr(lib, name)
            fn.restype = res
            fn.argtypes = args
        _lib = lib
    return _lib


def header_symbols(path: str = HEADER):
    """Names of the entry points declared in include/ibdl.h."""
    text = open(path).read()
    return sorted(set(re.findall(r"\b(ibdl_[a-z_]+)\s*\(", text)))


STAGES = ["spread", "fft_x_fwd", "fft_y_fwd", "fused_last_axis", "fft_y_inv", "fft_x_inv", "interp",
          "krylov", "fill"]


class IBDLError(RuntimeError):
    def __init__(self, status, message):
        super().__init__(f"{STATUS.get(status, status)}: {message}")
        self.status = status


def check_batch(status, handle=None):
    if status < 0:
        msg = load().ibdl_batch_last_error(handle)
        raise IBDLError(status, msg.decode() if msg else "")
    return status


def check(status, handle=None):
    if status < 0:
        msg = load().ibdl_last_error(handle)
        raise IBDLError(status, msg.decode() if msg else "")
    return status
