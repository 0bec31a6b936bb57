"""ctypes binding of libfrobinv (include/frobinv.h).

Argument marshalling only: every entry point forwards device pointers, sizes
and leading dimensions to the C ABI, which runs all arithmetic in HIP kernels.
PyTorch supplies device memory and the stream.  There is no fallback: if the
shared library is missing or fails to load, importing the binding raises.
"""
from __future__ import annotations

import ctypes
import os

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libfrobinv.so")
HEADER = os.path.join(os.path.dirname(HERE), "include", "frobinv.h")

FROB_OK = 0
FROB_SINGULAR = 1
FROB_NOT_HPD = 2
FROB_NO_CONVERGENCE = 3
FROB_E_ARG = -1
FROB_E_ALLOC = -2
FROB_E_HIP = -3
FROB_E_INTERNAL = -4
FROB_E_CAPTURE = -5

FROB_NEWTON_FROBENIUS = 0
FROB_NEWTON_COMPLEX_LU = 1
FROB_SHIFT_OFF = 0
FROB_SHIFT_AUTO = 1
FROB_SHIFT_ON = 2
FROB_SHIFT_PHASE = 3
FROB_SHIFT_COND = 4
FROB_PREC_F64 = 0
FROB_PREC_F32 = 1
FROB_PREC_BF16 = 2
FROB_REFINE_SKIP_FINAL_RESID = 1
FROB_REFINE_F32_CORRECTION = 2
FROB_REPORT_COND = 4


class frob_opts_t(ctypes.Structure):
    _fields_ = [("shift", ctypes.c_int), ("mu", ctypes.c_double), ("seed", ctypes.c_uint64),
                ("refine", ctypes.c_int), ("prec", ctypes.c_int), ("refine_tol", ctypes.c_double),
                ("refine_flags", ctypes.c_int), ("theta", ctypes.c_double), ("cond_tol", ctypes.c_double),
                ("panel", ctypes.c_int), ("reserved", ctypes.c_int)]


class frob_result_t(ctypes.Structure):
    _fields_ = [("info", ctypes.c_int), ("stage", ctypes.c_int), ("mu_used", ctypes.c_double),
                ("shifts_tried", ctypes.c_int), ("refine_steps", ctypes.c_int),
                ("resid0", ctypes.c_double), ("resid", ctypes.c_double), ("norm2_est", ctypes.c_double),
                ("cond1_C", ctypes.c_double), ("theta", ctypes.c_double)]

    def as_dict(self):
        return {"info": self.info, "stage": self.stage, "mu_used": self.mu_used,
                "shifts_tried": self.shifts_tried, "refine_steps": self.refine_steps,
                "resid0": self.resid0, "resid": self.resid, "norm2_est": self.norm2_est,
                "cond1_C": self.cond1_C, "theta": self.theta}


class frob_newton_opts_t(ctypes.Structure):
    _fields_ = [("tol", ctypes.c_double), ("max_iter", ctypes.c_int), ("inv", frob_opts_t), ("inverse", ctypes.c_int)]


class frob_newton_result_t(ctypes.Structure):
    _fields_ = [("iterations", ctypes.c_int), ("last_change", ctypes.c_double), ("inv", frob_result_t)]

    def as_dict(self):
        return {"iterations": self.iterations, "last_change": self.last_change, "inv": self.inv.as_dict()}


_vp = ctypes.c_void_p
_i = ctypes.c_int
_d = ctypes.c_double
_OPTS = ctypes.POINTER(frob_opts_t)
_RES = ctypes.POINTER(frob_result_t)

# name -> (restype, argtypes); kept in the order of include/frobinv.h
SIGNATURES = {
    "frob_default_opts": (None, [_OPTS]),
    "frob_create": (_i, [ctypes.POINTER(_vp), _i]),
    "frob_destroy": (_i, [_vp]),
    "frob_set_stream": (_i, [_vp, _vp]),
    "frob_workspace_bytes": (ctypes.c_size_t, [_vp]),
    "frob_inv_general": (_i, [_vp, _i, _vp, _i, _vp, _i, _vp, _vp, _i, _OPTS, _RES]),
    "frob_inv_hpd": (_i, [_vp, _i, _vp, _i, _vp, _i, _vp, _vp, _i, _OPTS, _RES]),
    "frob_inv_spd_pair": (_i, [_vp, _i, _vp, _i, _vp, _i, _vp, _vp, _i, _OPTS, _RES]),
    "frob_solve": (_i, [_vp, _i, _i, _vp, _i, _vp, _i, _vp, _vp, _i, _vp, _vp, _i, _OPTS, _RES]),
    "frob_inv_general_f32": (_i, [_vp, _i, _vp, _i, _vp, _i, _vp, _vp, _i, _OPTS, _RES]),
    "frob_inv_hpd_f32": (_i, [_vp, _i, _vp, _i, _vp, _i, _vp, _vp, _i, _OPTS, _RES]),
    "frob_solve_f32": (_i, [_vp, _i, _i, _vp, _i, _vp, _i, _vp, _vp, _i, _vp, _vp, _i, _OPTS, _RES]),
    "frob_refine": (_i, [_vp, _i, _vp, _i, _vp, _i, _vp, _vp, _i, _OPTS, _RES]),
    "frob_inv_tower": (_i, [_vp, _i, _i, ctypes.POINTER(_d), ctypes.POINTER(_vp), _i, ctypes.POINTER(_vp), _i, _OPTS,
                            _RES]),
    "frob_default_newton_opts": (None, [ctypes.POINTER(frob_newton_opts_t)]),
    "frob_sign": (_i, [_vp, _i, _vp, _vp, _i, _vp, _vp, _i, ctypes.POINTER(frob_newton_opts_t),
                       ctypes.POINTER(frob_newton_result_t)]),
    "frob_polar": (_i, [_vp, _i, _vp, _vp, _i, _vp, _vp, _i, _vp, _vp, _i, ctypes.POINTER(frob_newton_opts_t),
                        ctypes.POINTER(frob_newton_result_t)]),
    "frob_sylvester": (_i, [_vp, _i, _i, _vp, _vp, _i, _vp, _vp, _i, _vp, _vp, _i, _vp, _vp, _i,
                            ctypes.POINTER(frob_newton_opts_t), ctypes.POINTER(frob_newton_result_t)]),
    "frob_lyapunov": (_i, [_vp, _i, _vp, _vp, _i, _vp, _vp, _i, _vp, _vp, _i, ctypes.POINTER(frob_newton_opts_t),
                           ctypes.POINTER(frob_newton_result_t)]),
    "frob_cinv_lu": (_i, [_vp, _i, _vp, _vp, _i, _vp, _vp, _i, _i, _RES]),
    "frob_cinv_chol": (_i, [_vp, _i, _vp, _vp, _i, _vp, _vp, _i, _i, _RES]),
    "frob_inv_adjoint": (_i, [_vp, _i, _i, _i, _vp, _vp, _vp, _vp, _vp, _vp]),
    "frob_inv_batched": (_i, [_vp, _i, _i, _vp, _vp, _vp, _vp, _vp, _vp, _vp, _i]),
    "frob_inv_batched_noalloc": (_i, [_vp, _i, _i, _vp, _vp, _vp, _vp, _vp, _vp, _vp, _i]),
    "frob_batched_tune": (_i, [_vp, _i, ctypes.POINTER(ctypes.c_int)]),
    "frob_profile_enable": (_i, [_vp, _i]),
    "frob_profile_read": (_i, [_vp, _i, ctypes.POINTER(ctypes.c_longlong), ctypes.POINTER(_d),
                               ctypes.POINTER(_d), ctypes.POINTER(_d)]),
    "frob_status_string": (ctypes.c_char_p, [_i]),
}

_lib = None


def load(path: str = LIB_PATH):
    """Load libfrobinv.so and declare the C ABI.  Raises if it is missing."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(path):
        raise ImportError(f"libfrobinv.so not built at {path}; run paper_2208_01239_amd/build.py")
    # PyTorch ships its own HIP runtime (same SONAME as ROCm's).  Load it first so
    # the library binds to that single runtime instead of a second copy.
    import torch  # noqa: F401
    lib = ctypes.CDLL(path)
    for name, (res, args) in SIGNATURES.items():
        fn = getattr(lib, name)
        fn.restype = res
        fn.argtypes = args
    _lib = lib
    return lib


class FrobError(RuntimeError):
    def __init__(self, status: int, where: str, result: frob_result_t | None = None):
        name = load().frob_status_string(status).decode()
        super().__init__(f"{where}: {name}" + (f" {result.as_dict()}" if result is not None else ""))
        self.status = status
        self.result = result


class FrobSingularError(FrobError):
    pass


class FrobNotHPDError(FrobError):
    pass


class FrobNoConvergenceError(FrobError):
    """Newton-Schulz refinement cannot converge (||I - M X||_2 estimated >= 1, or the residual grew); X is unrefined."""


def check(status: int, where: str, result: frob_result_t | None = None):
    if status == FROB_OK:
        return
    if status == FROB_SINGULAR:
        raise FrobSingularError(status, where, result)
    if status == FROB_NOT_HPD:
        raise FrobNotHPDError(status, where, result)
    if status == FROB_NO_CONVERGENCE:
        raise FrobNoConvergenceError(status, where, result)
    raise FrobError(status, where, result)
