"""FP64 CPU oracle for Frobenius inversion (arXiv 2208.01239).

TEST INFRASTRUCTURE ONLY.  Only ``tests/``, ``__graft_entry__.smoke()`` and the
``cpu_baseline`` leg of ``bench.py`` may import this package.  The product
library never links, loads or calls it, and shares no code with it.

Thin ctypes wrapper over ``liboracle.so`` (plain C, see ``frob_oracle.c``).
Every routine takes real numpy arrays (the real and imaginary parts of the
complex input) and returns new arrays; ``info`` follows the C return codes.
"""
from __future__ import annotations

import ctypes
import os

import numpy as np

from . import build as _build

STAGE_A = 1000000
STAGE_C = 2000000

_HERE = os.path.dirname(os.path.abspath(__file__))
_LIB_PATH = os.path.join(_HERE, "liboracle.so")
_lib = None

_dp = ctypes.POINTER(ctypes.c_double)
_ip = ctypes.POINTER(ctypes.c_int)


def _load():
    global _lib
    if _lib is not None:
        return _lib
    src = os.path.join(_HERE, "frob_oracle.c")
    if not os.path.exists(_LIB_PATH) or os.path.getmtime(_LIB_PATH) < os.path.getmtime(src):
        _build.build()
    lib = ctypes.CDLL(_LIB_PATH)
    i, d = ctypes.c_int, ctypes.c_double
    lib.orc_cinv_lu.argtypes = [i, _dp, _dp, _dp, _dp, _ip, _dp]
    lib.orc_cinv_gj.argtypes = [i, _dp, _dp, _dp, _dp]
    lib.orc_frob_lu.argtypes = [i, _dp, _dp, _dp, _dp, _dp]
    lib.orc_frob_shift.argtypes = [i, _dp, _dp, d, _dp, _dp, _dp]
    lib.orc_frob_chol.argtypes = [i, _dp, _dp, _dp, _dp, _dp]
    lib.orc_cinv_chol.argtypes = [i, _dp, _dp, _dp, _dp, _dp]
    lib.orc_frob_solve.argtypes = [i, i, _dp, _dp, _dp, _dp, _dp, _dp, _dp]
    lib.orc_adjoint.argtypes = [i, _dp, _dp, _dp, _dp, _dp, _dp]
    lib.orc_adjoint.restype = None
    lib.orc_cmatmul.argtypes = [i, i, i, _dp, _dp, _dp, _dp, _dp, _dp]
    lib.orc_cmatmul.restype = None
    lib.orc_frob_chol_spd_pair.argtypes = [i, _dp, _dp, _dp, _dp, _dp]
    lib.orc_csolve_refined.argtypes = [i, i, _dp, _dp, _dp, _dp, i, _dp, _dp, _dp]
    lib.orc_csolve_refined.restype = ctypes.c_int
    lib.orc_tower_mul.argtypes = [i, i, _dp, _dp, _dp, _dp]
    lib.orc_tower_mul.restype = None
    lib.orc_tower_inv.argtypes = [i, i, _dp, _dp, _dp]
    lib.orc_tower_inv.restype = ctypes.c_int
    lib.orc_sign_newton.argtypes = [i, _dp, _dp, d, i, _dp, _dp, _ip]
    lib.orc_polar_newton.argtypes = [i, _dp, _dp, d, i, _dp, _dp, _dp, _dp, _ip]
    lib.orc_sylvester_newton.argtypes = [i, i, _dp, _dp, _dp, _dp, _dp, _dp, d, i, _dp, _dp, _ip]
    lib.orc_num_threads.argtypes = []
    lib.orc_set_num_threads.argtypes = [ctypes.c_int]
    for name in ("orc_cinv_lu", "orc_cinv_gj", "orc_frob_lu", "orc_frob_shift", "orc_frob_chol",
                 "orc_cinv_chol", "orc_frob_solve", "orc_num_threads", "orc_set_num_threads", "orc_sign_newton", "orc_frob_chol_spd_pair",
                 "orc_polar_newton", "orc_sylvester_newton"):
        getattr(lib, name).restype = ctypes.c_int
    _lib = lib
    return lib


def _c(a):
    a = np.ascontiguousarray(a, dtype=np.float64)
    return a, a.ctypes.data_as(_dp)


def _out(*shape):
    a = np.zeros(shape, dtype=np.float64)
    return a, a.ctypes.data_as(_dp)


def num_threads() -> int:
    return _load().orc_num_threads()


def set_num_threads(t: int) -> int:
    """Threads of later calls (timing only); returns the previous count."""
    return _load().orc_set_num_threads(int(t))


def cinv_lu(Mr, Mi):
    """Algorithm 4 in complex arithmetic.  Returns (Xr, Xi, info, piv, flops)."""
    lib = _load()
    n = Mr.shape[0]
    (Mr, pr), (Mi, pi) = _c(Mr), _c(Mi)
    (Xr, xr), (Xi, xi) = _out(n, n), _out(n, n)
    piv = np.zeros(n, dtype=np.int32)
    fl = ctypes.c_double(0)
    info = lib.orc_cinv_lu(n, pr, pi, xr, xi, piv.ctypes.data_as(_ip), ctypes.byref(fl))
    return Xr, Xi, info, piv, fl.value


def cinv_gj(Mr, Mi):
    """Gauss-Jordan on [M | I].  Returns (Xr, Xi, info)."""
    lib = _load()
    n = Mr.shape[0]
    (Mr, pr), (Mi, pi) = _c(Mr), _c(Mi)
    (Xr, xr), (Xi, xi) = _out(n, n), _out(n, n)
    info = lib.orc_cinv_gj(n, pr, pi, xr, xi)
    return Xr, Xi, info


def frob_lu(A, B):
    """Algorithm 5.  Returns (Xr, Xi, info, flops)."""
    lib = _load()
    n = A.shape[0]
    (A, pa), (B, pb) = _c(A), _c(B)
    (Xr, xr), (Xi, xi) = _out(n, n), _out(n, n)
    fl = ctypes.c_double(0)
    info = lib.orc_frob_lu(n, pa, pb, xr, xi, ctypes.byref(fl))
    return Xr, Xi, info, fl.value


def frob_shift(A, B, mu):
    """Algorithm 6 with the given shift mu.  Returns (Xr, Xi, info, flops)."""
    lib = _load()
    n = A.shape[0]
    (A, pa), (B, pb) = _c(A), _c(B)
    (Xr, xr), (Xi, xi) = _out(n, n), _out(n, n)
    fl = ctypes.c_double(0)
    info = lib.orc_frob_shift(n, pa, pb, float(mu), xr, xi, ctypes.byref(fl))
    return Xr, Xi, info, fl.value


def frob_chol(A, B):
    """Algorithm 7 (HPD input).  Returns (Xr, Xi, info, flops)."""
    lib = _load()
    n = A.shape[0]
    (A, pa), (B, pb) = _c(A), _c(B)
    (Xr, xr), (Xi, xi) = _out(n, n), _out(n, n)
    fl = ctypes.c_double(0)
    info = lib.orc_frob_chol(n, pa, pb, xr, xi, ctypes.byref(fl))
    return Xr, Xi, info, fl.value


def frob_chol_spd_pair(A, B):
    """Algorithm 7 with step 5 X4 = A + X3 (A, B symmetric positive definite).
    Returns (Xr, Xi, info, flops)."""
    lib = _load()
    n = A.shape[0]
    (A, pa), (B, pb) = _c(A), _c(B)
    (Xr, xr), (Xi, xi) = _out(n, n), _out(n, n)
    fl = ctypes.c_double(0)
    info = lib.orc_frob_chol_spd_pair(n, pa, pb, xr, xi, ctypes.byref(fl))
    return Xr, Xi, info, fl.value


def cinv_chol(Mr, Mi):
    """Algorithm 8 in complex arithmetic.  Returns (Xr, Xi, info, flops)."""
    lib = _load()
    n = Mr.shape[0]
    (Mr, pr), (Mi, pi) = _c(Mr), _c(Mi)
    (Xr, xr), (Xi, xi) = _out(n, n), _out(n, n)
    fl = ctypes.c_double(0)
    info = lib.orc_cinv_chol(n, pr, pi, xr, xi, ctypes.byref(fl))
    return Xr, Xi, info, fl.value


def frob_solve(A, B, c, d):
    """Algorithm 3 (sign of step 7 corrected) for n x p right-hand sides.
    Returns (x, y, info, flops)."""
    lib = _load()
    n = A.shape[0]
    c = np.asarray(c, dtype=np.float64)
    d = np.asarray(d, dtype=np.float64)
    squeeze = c.ndim == 1
    if squeeze:
        c, d = c[:, None], d[:, None]
    p = c.shape[1]
    (A, pa), (B, pb), (c, pc), (d, pd) = _c(A), _c(B), _c(c), _c(d)
    (x, px), (y, py) = _out(n, p), _out(n, p)
    fl = ctypes.c_double(0)
    info = lib.orc_frob_solve(n, p, pa, pb, pc, pd, px, py, ctypes.byref(fl))
    if squeeze:
        x, y = x[:, 0], y[:, 0]
    return x, y, info, fl.value


def adjoint(Xr, Xi, Gr, Gi):
    """dM = -X^H G X^H.  Returns (dMr, dMi)."""
    lib = _load()
    n = Xr.shape[0]
    (Xr, a), (Xi, b), (Gr, c), (Gi, d) = _c(Xr), _c(Xi), _c(Gr), _c(Gi)
    (R, pr), (I, pi) = _out(n, n), _out(n, n)
    lib.orc_adjoint(n, a, b, c, d, pr, pi)
    return R, I


def cmatmul(Xr, Xi, Yr, Yi):
    """Plain complex product (X Y).  Returns (Zr, Zi)."""
    lib = _load()
    n, k = Xr.shape
    k2, m = Yr.shape
    assert k == k2
    (Xr, a), (Xi, b), (Yr, c), (Yi, d) = _c(Xr), _c(Xi), _c(Yr), _c(Yi)
    (Zr, pr), (Zi, pi) = _out(n, m), _out(n, m)
    lib.orc_cmatmul(n, k, m, a, b, c, d, pr, pi)
    return Zr, Zi


def sign_newton(Xr, Xi, eps=1e-3, kmax=100):
    """Matrix sign by the Newton iteration of Section 5.3.  Returns (Sr, Si, info, iters)."""
    lib = _load()
    n = Xr.shape[0]
    (Xr, a), (Xi, b) = _c(Xr), _c(Xi)
    (Sr, pr), (Si, pi) = _out(n, n), _out(n, n)
    it = ctypes.c_int(0)
    info = lib.orc_sign_newton(n, a, b, float(eps), int(kmax), pr, pi, ctypes.byref(it))
    return Sr, Si, info, it.value


def polar_newton(Xr, Xi, eps=1e-3, kmax=100):
    """Polar decomposition X = Q P by the Newton iteration of Section 5.5.
    Returns (Qr, Qi, Pr, Pi, info, iters)."""
    lib = _load()
    n = Xr.shape[0]
    (Xr, a), (Xi, b) = _c(Xr), _c(Xi)
    (Qr, qr), (Qi, qi), (Pr, pr), (Pi, pi) = _out(n, n), _out(n, n), _out(n, n), _out(n, n)
    it = ctypes.c_int(0)
    info = lib.orc_polar_newton(n, a, b, float(eps), int(kmax), qr, qi, pr, pi, ctypes.byref(it))
    return Qr, Qi, Pr, Pi, info, it.value


def sylvester_newton(Ar, Ai, Br, Bi, Cr, Ci, eps=1e-1, kmax=100):
    """A Y + Y B = C through the sign of [[A, -C], [0, -B]] (Section 5.4).
    Returns (Yr, Yi, info, iters)."""
    lib = _load()
    p, q = Ar.shape[0], Br.shape[0]
    (Ar, a1), (Ai, a2), (Br, b1), (Bi, b2), (Cr, c1), (Ci, c2) = (_c(x) for x in (Ar, Ai, Br, Bi, Cr, Ci))
    (Yr, yr), (Yi, yi) = _out(p, q), _out(p, q)
    it = ctypes.c_int(0)
    info = lib.orc_sylvester_newton(p, q, a1, a2, b1, b2, c1, c2, float(eps), int(kmax), yr, yi, ctypes.byref(it))
    return Yr, Yi, info, it.value


def tower_mul(tau, X, Y):
    """Product in F_m^{n x n} (Section 2.4); X, Y: (2^m, n, n) coefficient planes."""
    lib = _load()
    tau = np.ascontiguousarray(tau, dtype=np.float64)
    m, n = len(tau), X.shape[1]
    (X, px), (Y, py), (t, pt) = _c(X), _c(Y), _c(tau)
    Z, pz = _out(1 << m, n, n)
    lib.orc_tower_mul(m, n, pt, px, py, pz)
    return Z


def tower_inv(tau, C):
    """Inverse in F_m^{n x n} through the regular representation.  Returns (Xinv planes, info)."""
    lib = _load()
    tau = np.ascontiguousarray(tau, dtype=np.float64)
    m, n = len(tau), C.shape[1]
    (C, pc), (t, pt) = _c(C), _c(tau)
    X, px = _out(1 << m, n, n)
    info = lib.orc_tower_inv(m, n, pt, pc, px)
    return X, info


def csolve_refined(Mr, Mi, Br, Bi, steps=3):
    """x = M^{-1} b for n x p right-hand sides: complex GEPP plus refinement with
    double-double residuals.  Returns (Xr, Xi, info, last) with last the
    largest relative max-norm size of the final correction over the columns."""
    lib = _load()
    n = Mr.shape[0]
    Br = np.asarray(Br, dtype=np.float64)
    Bi = np.asarray(Bi, dtype=np.float64)
    if Br.ndim == 1:
        Br, Bi = Br[:, None], Bi[:, None]
    p = Br.shape[1]
    (Mr, a), (Mi, b), (Br, c), (Bi, d) = _c(Mr), _c(Mi), _c(Br), _c(Bi)
    (Xr, xr), (Xi, xi) = _out(n, p), _out(n, p)
    last = ctypes.c_double(0.0)
    info = lib.orc_csolve_refined(n, p, a, b, c, d, int(steps), xr, xi, ctypes.byref(last))
    return Xr, Xi, info, last.value
