"""Frobenius inversion of complex matrices with real operations on AMD MI355X.

Python binding of libfrobinv (C ABI in ``include/frobinv.h``).  The functions
below carry the names of the C entry points and only marshal arguments: torch
tensors provide device memory and the current stream; all arithmetic runs in
the library's HIP kernels.  Importing this package does not load the library;
the first call does, and raises if it is missing (there is no fallback path).

Tensors: float64 (or float32 for the FP32-storage twins of the single-matrix
calls), on a ROCm device, row-major with unit column stride (a leading
dimension ``stride(0) >= n`` is allowed).
"""
from __future__ import annotations

import ctypes

from . import _lib
from ._lib import (FROB_NEWTON_COMPLEX_LU, FROB_NEWTON_FROBENIUS,  # noqa: F401
                   FROB_PREC_BF16, FROB_PREC_F32, FROB_PREC_F64, FROB_REFINE_F32_CORRECTION,
                   FROB_REFINE_SKIP_FINAL_RESID, FROB_REPORT_COND, FROB_SHIFT_COND, FROB_SHIFT_PHASE,
                   FROB_SHIFT_AUTO, FROB_SHIFT_OFF, FROB_SHIFT_ON, FrobError, FrobNoConvergenceError, FrobNotHPDError, FrobSingularError,
                   frob_opts_t, frob_result_t)

__all__ = ["Handle", "frob_inv_general", "frob_inv_hpd", "frob_solve", "frob_refine", "frob_cinv_lu", "frob_cinv_chol",
           "frob_inv_adjoint", "frob_inv_batched", "frob_batched_tune", "BatchedPlan",
           "FrobError", "FrobSingularError", "FrobNotHPDError", "FrobNoConvergenceError", "FROB_SHIFT_OFF",
           "FROB_SHIFT_AUTO", "FROB_SHIFT_ON", "FROB_NEWTON_FROBENIUS", "FROB_NEWTON_COMPLEX_LU", "FROB_PREC_F64", "FROB_PREC_F32", "FROB_PREC_BF16",
           "FROB_REFINE_SKIP_FINAL_RESID", "FROB_REFINE_F32_CORRECTION", "load_library", "frob_sign", "frob_polar",
           "frob_sylvester", "frob_lyapunov", "frob_inv_spd_pair", "frob_inv_tower"]


def load_library():
    return _lib.load()


class Handle:
    """Owns a frob_handle_t on one device (workspace, status words, stream)."""

    def __init__(self, device: int = 0):
        lib = _lib.load()
        h = ctypes.c_void_p()
        _lib.check(lib.frob_create(ctypes.byref(h), int(device)), "frob_create")
        self._h = h
        self.device = int(device)

    @property
    def ptr(self):
        if self._h is None:
            raise RuntimeError("handle closed")
        return self._h

    def close(self):
        if getattr(self, "_h", None) is not None:
            _lib.load().frob_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()

    def workspace_bytes(self) -> int:
        return int(_lib.load().frob_workspace_bytes(self.ptr))

    def profile(self, on: bool = True):
        """Enable (and reset) or disable HIP-event timing of kernel classes."""
        _lib.check(_lib.load().frob_profile_enable(self.ptr, 1 if on else 0), "frob_profile_enable")

    def profile_read(self, kernel_class: int = 0):
        """(launches, total_ms, flops, bytes) accumulated for a kernel class."""
        n, ms, fl, by = ctypes.c_longlong(), ctypes.c_double(), ctypes.c_double(), ctypes.c_double()
        _lib.check(_lib.load().frob_profile_read(self.ptr, int(kernel_class), ctypes.byref(n), ctypes.byref(ms),
                                                 ctypes.byref(fl), ctypes.byref(by)), "frob_profile_read")
        return int(n.value), float(ms.value), float(fl.value), float(by.value)

    def bind_stream(self, stream=None):
        import torch
        s = stream if stream is not None else torch.cuda.current_stream(self.device)
        _lib.check(_lib.load().frob_set_stream(self.ptr, ctypes.c_void_p(s.cuda_stream)), "frob_set_stream")


def _mat(t, n_rows, n_cols, name, dtype=None):
    import torch
    dtype = dtype or torch.float64
    if not isinstance(t, torch.Tensor) or t.dtype != dtype or t.device.type != "cuda":
        raise TypeError(f"{name}: expected a {dtype} tensor on a ROCm device")
    if t.dim() != 2 or t.shape[0] != n_rows or t.shape[1] != n_cols:
        raise ValueError(f"{name}: expected shape ({n_rows}, {n_cols}), got {tuple(t.shape)}")
    # strides of extent-1 dimensions do not address anything
    cs = 1 if n_cols == 1 else t.stride(1)
    ld = n_cols if n_rows == 1 else t.stride(0)
    if cs != 1 or ld < n_cols:
        raise ValueError(f"{name}: rows must be contiguous with leading dimension >= {n_cols}")
    return ctypes.c_void_p(t.data_ptr()), int(ld)


def _opts(shift, mu, seed, refine, prec=0, refine_tol=0.0, final_resid=True, f32_correction=False, theta=0.0,
          cond_tol=0.0, report_cond=False, panel=0):
    o = frob_opts_t()
    _lib.load().frob_default_opts(ctypes.byref(o))
    o.shift = int(shift)
    o.mu = float(mu)
    o.seed = int(seed)
    o.refine = int(refine)
    o.prec = int(prec)
    o.refine_tol = float(refine_tol)
    o.refine_flags = (0 if final_resid else FROB_REFINE_SKIP_FINAL_RESID) | \
        (FROB_REFINE_F32_CORRECTION if f32_correction else 0) | (FROB_REPORT_COND if report_cond else 0)
    o.theta = float(theta)
    o.cond_tol = float(cond_tol)
    o.panel = int(panel)
    return o


def _empty_like_sq(A, n):
    import torch
    return torch.empty((n, n), dtype=A.dtype, device=A.device)


def _fn32(name, A):
    """The FP64 entry point, or its FP32-storage twin for float32 operands."""
    import torch
    return (name + "_f32", torch.float32) if A.dtype == torch.float32 else (name, torch.float64)


def frob_inv_general(h: Handle, A, B, Xr=None, Xi=None, *, shift=FROB_SHIFT_AUTO, mu=0.0, seed=0, refine=0,
                     prec=FROB_PREC_F64, refine_tol=0.0, final_resid=True, f32_correction=False, theta=0.0,
                     cond_tol=0.0, report_cond=False, panel=0):
    """(A + iB)^{-1} = Xr + i Xi by Algorithm 5 (and 6 when shifting).

    prec: operand precision of the matrix-core products (FROB_PREC_F64/F32/BF16);
    refine: maximum number of Newton-Schulz steps (residual formed in FP64);
    final_resid=False: skip the residual of the returned inverse when the step
    limit ends refinement (result "resid" is then NaN);
    f32_correction=True: after FP64 factorizations, form each step's
    correction X R with FP32 matrix-core operands (the residual stays FP64);
    shift=FROB_SHIFT_PHASE with theta: invert e^{i theta} M and rotate back
    (theta = -pi/2: the formula for invertible B); shift=FROB_SHIFT_COND:
    rotations tried until u kappa_1(C) <= cond_tol; report_cond: kappa_1(C)
    in the result; panel: panel width of the look-ahead LUs (0 = 64; 16, 32,
    48 or 64) from order 1024."""
    n = A.shape[0]
    name, dt = _fn32("frob_inv_general", A)
    Xr = _empty_like_sq(A, n) if Xr is None else Xr
    Xi = _empty_like_sq(A, n) if Xi is None else Xi
    pa, lda = _mat(A, n, n, "A", dt)
    pb, ldb = _mat(B, n, n, "B", dt)
    pr, ldx = _mat(Xr, n, n, "Xr", dt)
    pi, ldxi = _mat(Xi, n, n, "Xi", dt)
    if ldx != ldxi:
        raise ValueError("Xr and Xi must share a leading dimension")
    h.bind_stream()
    o, r = _opts(shift, mu, seed, refine, prec, refine_tol, final_resid, f32_correction, theta, cond_tol,
                 report_cond, panel), frob_result_t()
    st = getattr(_lib.load(), name)(h.ptr, n, pa, lda, pb, ldb, pr, pi, ldx, ctypes.byref(o), ctypes.byref(r))
    _lib.check(st, name, r)
    return Xr, Xi, r.as_dict()


def frob_inv_hpd(h: Handle, A, B, Xr=None, Xi=None, *, refine=0, prec=FROB_PREC_F64, refine_tol=0.0,
                 final_resid=True, f32_correction=False):
    """(A + iB)^{-1} for Hermitian positive definite A + iB (Algorithm 7)."""
    n = A.shape[0]
    name, dt = _fn32("frob_inv_hpd", A)
    Xr = _empty_like_sq(A, n) if Xr is None else Xr
    Xi = _empty_like_sq(A, n) if Xi is None else Xi
    pa, lda = _mat(A, n, n, "A", dt)
    pb, ldb = _mat(B, n, n, "B", dt)
    pr, ldx = _mat(Xr, n, n, "Xr", dt)
    pi, ldxi = _mat(Xi, n, n, "Xi", dt)
    if ldx != ldxi:
        raise ValueError("Xr and Xi must share a leading dimension")
    h.bind_stream()
    o, r = _opts(FROB_SHIFT_OFF, 0.0, 0, refine, prec, refine_tol, final_resid, f32_correction), frob_result_t()
    st = getattr(_lib.load(), name)(h.ptr, n, pa, lda, pb, ldb, pr, pi, ldx, ctypes.byref(o), ctypes.byref(r))
    _lib.check(st, name, r)
    return Xr, Xi, r.as_dict()


def frob_inv_spd_pair(h: Handle, A, B, Xr=None, Xi=None, *, refine=0, prec=FROB_PREC_F64, refine_tol=0.0,
                      final_resid=True, f32_correction=False):
    """(A + iB)^{-1} for A, B symmetric positive definite (Algorithm 7 with C = A + X1^T X1)."""
    n = A.shape[0]
    Xr = _empty_like_sq(A, n) if Xr is None else Xr
    Xi = _empty_like_sq(A, n) if Xi is None else Xi
    pa, lda = _mat(A, n, n, "A")
    pb, ldb = _mat(B, n, n, "B")
    pr, ldx = _mat(Xr, n, n, "Xr")
    pi, ldxi = _mat(Xi, n, n, "Xi")
    if ldx != ldxi:
        raise ValueError("Xr and Xi must share a leading dimension")
    h.bind_stream()
    o, r = _opts(FROB_SHIFT_OFF, 0.0, 0, refine, prec, refine_tol, final_resid, f32_correction), frob_result_t()
    st = _lib.load().frob_inv_spd_pair(h.ptr, n, pa, lda, pb, ldb, pr, pi, ldx, ctypes.byref(o), ctypes.byref(r))
    _lib.check(st, "frob_inv_spd_pair", r)
    return Xr, Xi, r.as_dict()


def frob_refine(h: Handle, A, B, Xr, Xi, *, refine=4, prec=FROB_PREC_F64, refine_tol=0.0, final_resid=True,
                f32_correction=False):
    """Newton-Schulz refinement, in place, of an approximate inverse Xr + i Xi of A + iB.

    Raises FrobNoConvergenceError (X left unchanged) when ||I - M X||_2 is
    estimated >= 1 or the residual grows.  Returns the result dict."""
    n = A.shape[0]
    pa, lda = _mat(A, n, n, "A")
    pb, ldb = _mat(B, n, n, "B")
    pr, ldx = _mat(Xr, n, n, "Xr")
    pi, ldxi = _mat(Xi, n, n, "Xi")
    if ldx != ldxi:
        raise ValueError("Xr and Xi must share a leading dimension")
    h.bind_stream()
    o, r = _opts(FROB_SHIFT_OFF, 0.0, 0, refine, prec, refine_tol, final_resid, f32_correction), frob_result_t()
    st = _lib.load().frob_refine(h.ptr, n, pa, lda, pb, ldb, pr, pi, ldx, ctypes.byref(o), ctypes.byref(r))
    _lib.check(st, "frob_refine", r)
    return r.as_dict()


def frob_solve(h: Handle, A, B, c, d, x=None, y=None, *, shift=FROB_SHIFT_AUTO, mu=0.0, seed=0, panel=0):
    """Solve (A + iB)(x + iy) = c + id for n x p right-hand sides (Algorithm 3).
    float32 operands use the FP32-storage twin (FP64 arithmetic); panel as
    for frob_inv_general."""
    import torch
    n = A.shape[0]
    p = c.shape[1]
    name, dt = _fn32("frob_solve", A)
    x = torch.empty((n, p), dtype=dt, device=A.device) if x is None else x
    y = torch.empty((n, p), dtype=dt, device=A.device) if y is None else y
    pa, lda = _mat(A, n, n, "A", dt)
    pb, ldb = _mat(B, n, n, "B", dt)
    pc, ldc = _mat(c, n, p, "c", dt)
    pd, ldd = _mat(d, n, p, "d", dt)
    px, ldx = _mat(x, n, p, "x", dt)
    py, ldy = _mat(y, n, p, "y", dt)
    if ldc != ldd or ldx != ldy:
        raise ValueError("c/d and x/y must share leading dimensions")
    h.bind_stream()
    o, r = _opts(shift, mu, seed, 0, panel=panel), frob_result_t()
    st = getattr(_lib.load(), name)(h.ptr, n, p, pa, lda, pb, ldb, pc, pd, ldc, px, py, ldx, ctypes.byref(o),
                                    ctypes.byref(r))
    _lib.check(st, name, r)
    return x, y, r.as_dict()


def _cinv(fn_name, h, Mr, Mi, Xr, Xi, form):
    n = Mr.shape[0]
    Xr = _empty_like_sq(Mr, n) if Xr is None else Xr
    Xi = _empty_like_sq(Mr, n) if Xi is None else Xi
    pr, ldm = _mat(Mr, n, n, "Mr")
    pi, ldmi = _mat(Mi, n, n, "Mi")
    qr, ldx = _mat(Xr, n, n, "Xr")
    qi, ldxi = _mat(Xi, n, n, "Xi")
    if ldm != ldmi or ldx != ldxi:
        raise ValueError("planar pairs must share a leading dimension")
    h.bind_stream()
    r = frob_result_t()
    st = getattr(_lib.load(), fn_name)(h.ptr, n, pr, pi, ldm, qr, qi, ldx, int(form), ctypes.byref(r))
    _lib.check(st, fn_name, r)
    return Xr, Xi, r.as_dict()


def frob_cinv_lu(h: Handle, Mr, Mi, Xr=None, Xi=None, *, form=1):
    """Baseline: complex-arithmetic LU inversion (Algorithm 4; form 0 as printed, 1 getri style)."""
    return _cinv("frob_cinv_lu", h, Mr, Mi, Xr, Xi, form)


def frob_cinv_chol(h: Handle, Mr, Mi, Xr=None, Xi=None, *, form=1):
    """Baseline: complex-arithmetic Cholesky inversion (Algorithm 8; form 0 as printed, 1 potri style)."""
    return _cinv("frob_cinv_chol", h, Mr, Mi, Xr, Xi, form)


def _batch3(t, name, dtype=None):
    import torch
    if not isinstance(t, torch.Tensor) or t.device.type != "cuda" or t.dim() != 3:
        raise TypeError(f"{name}: expected a (batch, n, n) tensor on a ROCm device")
    if t.dtype not in (torch.float32, torch.float64) or (dtype is not None and t.dtype != dtype):
        raise TypeError(f"{name}: expected float32 or float64 matching the other operands")
    if t.shape[1] != t.shape[2] or not t.is_contiguous():
        raise ValueError(f"{name}: expected contiguous square matrices")
    return ctypes.c_void_p(t.data_ptr())


def frob_inv_adjoint(h: Handle, Xr, Xi, Gr, Gi, dMr=None, dMi=None):
    """dM = -X^H G X^H for a batch of matrices (reverse-mode derivative of M -> M^{-1}).

    All operands are (batch, n, n) contiguous float32 or float64 tensors; G is the
    gradient with respect to X in PyTorch's convention (dL/dRe X + i dL/dIm X)."""
    import torch
    dt = Xr.dtype
    b, n = Xr.shape[0], Xr.shape[1]
    dMr = torch.empty_like(Xr) if dMr is None else dMr
    dMi = torch.empty_like(Xr) if dMi is None else dMi
    ptrs = [_batch3(t, nm, dt) for t, nm in ((Xr, "Xr"), (Xi, "Xi"), (Gr, "Gr"), (Gi, "Gi"), (dMr, "dMr"),
                                              (dMi, "dMi"))]
    for t in (Xi, Gr, Gi, dMr, dMi):
        if t.shape != Xr.shape:
            raise ValueError("all operands must have the same shape")
    storage = FROB_PREC_F32 if dt == torch.float32 else FROB_PREC_F64
    h.bind_stream()
    st = _lib.load().frob_inv_adjoint(h.ptr, b, n, storage, *ptrs)
    _lib.check(st, "frob_inv_adjoint")
    return dMr, dMi


class BatchedPlan:
    """Device-side description of a batch for frob_inv_batched: per-matrix
    orders and kinds and the four pointer arrays, kept alive with the tensors
    they point to (so that a call can be repeated, or captured in a graph)."""

    def __init__(self, As, Bs, kinds, Xr=None, Xi=None):
        import torch
        if not (len(As) == len(Bs) == len(kinds)) or not As:
            raise ValueError("As, Bs and kinds must be non-empty and of equal length")
        dt = As[0].dtype
        if dt not in (torch.float32, torch.float64):
            raise TypeError("matrices must be float32 or float64")
        dev = As[0].device
        for t in list(As) + list(Bs):
            if t.dtype != dt or t.device != dev or t.dim() != 2 or t.shape[0] != t.shape[1] or not t.is_contiguous():
                raise ValueError("every matrix must be a contiguous square tensor of the batch's dtype and device")
        ns = [int(a.shape[0]) for a in As]
        if min(ns) < 1 or max(ns) > 512:
            raise ValueError("batched orders must lie in [1, 512]")
        if any(int(k) not in (0, 1) for k in kinds):
            raise ValueError("kinds must be 0 (general) or 1 (Hermitian positive definite)")
        for a, b in zip(As, Bs):
            if b.shape != a.shape:
                raise ValueError("A and B of a matrix must have the same order")
        self.As, self.Bs = list(As), list(Bs)
        self.Xr = [torch.empty_like(a) for a in As] if Xr is None else list(Xr)
        self.Xi = [torch.empty_like(a) for a in As] if Xi is None else list(Xi)
        self.count = len(As)
        self.nmax = max(ns)
        self.storage = FROB_PREC_F32 if dt == torch.float32 else FROB_PREC_F64

        def ptrs(ts):
            return torch.tensor([t.data_ptr() for t in ts], dtype=torch.int64, device=dev)

        self.n_dev = torch.tensor(ns, dtype=torch.int32, device=dev)
        self.kind_dev = torch.tensor([int(k) for k in kinds], dtype=torch.int32, device=dev)
        self.pA, self.pB, self.pXr, self.pXi = ptrs(self.As), ptrs(self.Bs), ptrs(self.Xr), ptrs(self.Xi)
        self.info_dev = torch.zeros(self.count, dtype=torch.int32, device=dev)

    def launch(self, h: "Handle", noalloc: bool = False):
        """Enqueue the batched inversion on the handle's stream (asynchronous).
        noalloc=True uses frob_inv_batched_noalloc (fixed device scratch, no allocation)."""
        h.bind_stream()
        vp = ctypes.c_void_p
        name = "frob_inv_batched_noalloc" if noalloc else "frob_inv_batched"
        st = getattr(_lib.load(), name)(h.ptr, self.count, self.nmax, vp(self.n_dev.data_ptr()),
                                         vp(self.kind_dev.data_ptr()), vp(self.pA.data_ptr()),
                                         vp(self.pB.data_ptr()), vp(self.pXr.data_ptr()),
                                         vp(self.pXi.data_ptr()), vp(self.info_dev.data_ptr()), self.storage)
        _lib.check(st, name)


def frob_inv_batched(h: Handle, As, Bs, kinds):
    """Invert a batch of uneven-order matrices in one persistent launch.

    kinds[i] = 0 (general, Algorithm 5) or 1 (Hermitian positive definite,
    Algorithm 7).  Returns (Xr list, Xi list, info numpy array)."""
    import torch
    plan = BatchedPlan(As, Bs, kinds)
    plan.launch(h)
    torch.cuda.current_stream().synchronize()
    return plan.Xr, plan.Xi, plan.info_dev.cpu().numpy()


def frob_batched_tune(h: Handle, storage=FROB_PREC_F64):
    """Autotune the batched panel widths; returns the table {(kind, class): nb}."""
    table = (ctypes.c_int * 8)()
    h.bind_stream()
    _lib.check(_lib.load().frob_batched_tune(h.ptr, int(storage), table), "frob_batched_tune")
    return {(k, c): table[4 * k + c] for k in range(2) for c in range(4)}


# ----------------------------------------------------------------- Newton iterations (Section 5)
def _newton_opts(tol, max_iter, **inv):
    """Options of a Newton driver; inverse=FROB_NEWTON_COMPLEX_LU takes every
    inverse from the complex-LU baseline instead of Frobenius inversion."""
    o = _lib.frob_newton_opts_t()
    _lib.load().frob_default_newton_opts(ctypes.byref(o))
    o.tol = float(tol)
    o.max_iter = int(max_iter)
    o.inverse = int(inv.pop("inverse", FROB_NEWTON_FROBENIUS))
    o.inv = _opts(inv.get("shift", FROB_SHIFT_AUTO), inv.get("mu", 0.0), inv.get("seed", 0), inv.get("refine", 0),
                  inv.get("prec", FROB_PREC_F64), inv.get("refine_tol", 0.0), inv.get("final_resid", True),
                  inv.get("f32_correction", False))
    return o


def frob_sign(h: Handle, Xr, Xi, Sr=None, Si=None, *, tol=1e-3, max_iter=100, **inv):
    """Matrix sign by Newton's iteration X <- (X + X^{-1}) / 2 (Section 5.3), every
    inverse by Frobenius inversion.  Returns (Sr, Si, result dict)."""
    n = Xr.shape[0]
    Sr = _empty_like_sq(Xr, n) if Sr is None else Sr
    Si = _empty_like_sq(Xr, n) if Si is None else Si
    px, ldx = _mat(Xr, n, n, "Xr")
    pxi, ldxi = _mat(Xi, n, n, "Xi")
    ps, lds = _mat(Sr, n, n, "Sr")
    psi, ldsi = _mat(Si, n, n, "Si")
    if ldx != ldxi or lds != ldsi:
        raise ValueError("planar pairs must share a leading dimension")
    h.bind_stream()
    o, r = _newton_opts(tol, max_iter, **inv), _lib.frob_newton_result_t()
    _lib.check(_lib.load().frob_sign(h.ptr, n, px, pxi, ldx, ps, psi, lds, ctypes.byref(o), ctypes.byref(r)),
               "frob_sign", r.inv)
    return Sr, Si, r.as_dict()


def frob_polar(h: Handle, Xr, Xi, *, tol=1e-3, max_iter=100, **inv):
    """Polar decomposition X = Q P by X <- (X + X^{-H}) / 2 (Section 5.5), P = Q^H X.
    Returns (Qr, Qi, Pr, Pi, result dict)."""
    n = Xr.shape[0]
    Qr, Qi, Pr, Pi = (_empty_like_sq(Xr, n) for _ in range(4))
    px, ldx = _mat(Xr, n, n, "Xr")
    pxi, ldxi = _mat(Xi, n, n, "Xi")
    if ldx != ldxi:
        raise ValueError("Xr and Xi must share a leading dimension")
    h.bind_stream()
    o, r = _newton_opts(tol, max_iter, **inv), _lib.frob_newton_result_t()
    vp = ctypes.c_void_p
    _lib.check(_lib.load().frob_polar(h.ptr, n, px, pxi, ldx, vp(Qr.data_ptr()), vp(Qi.data_ptr()), n,
                                      vp(Pr.data_ptr()), vp(Pi.data_ptr()), n, ctypes.byref(o), ctypes.byref(r)),
               "frob_polar", r.inv)
    return Qr, Qi, Pr, Pi, r.as_dict()


def frob_sylvester(h: Handle, Ar, Ai, Br, Bi, Cr, Ci, *, tol=1e-1, max_iter=100, **inv):
    """A Y + Y B = C through the sign of [[A, -C], [0, -B]] (Section 5.4).
    Returns (Yr, Yi, result dict)."""
    import torch
    p, q = Ar.shape[0], Br.shape[0]
    Yr = torch.empty((p, q), dtype=torch.float64, device=Ar.device)
    Yi = torch.empty_like(Yr)
    pa, lda = _mat(Ar, p, p, "Ar"); pai, ldai = _mat(Ai, p, p, "Ai")
    pb, ldb = _mat(Br, q, q, "Br"); pbi, ldbi = _mat(Bi, q, q, "Bi")
    pc, ldc = _mat(Cr, p, q, "Cr"); pci, ldci = _mat(Ci, p, q, "Ci")
    if lda != ldai or ldb != ldbi or ldc != ldci:
        raise ValueError("planar pairs must share a leading dimension")
    h.bind_stream()
    o, r = _newton_opts(tol, max_iter, **inv), _lib.frob_newton_result_t()
    vp = ctypes.c_void_p
    _lib.check(_lib.load().frob_sylvester(h.ptr, p, q, pa, pai, lda, pb, pbi, ldb, pc, pci, ldc, vp(Yr.data_ptr()),
                                          vp(Yi.data_ptr()), q, ctypes.byref(o), ctypes.byref(r)),
               "frob_sylvester", r.inv)
    return Yr, Yi, r.as_dict()


def frob_lyapunov(h: Handle, Ar, Ai, Cr, Ci, *, tol=1e-1, max_iter=100, **inv):
    """A Y + Y A^H = C (Section 5.4 with B = A^H).  Returns (Yr, Yi, result dict)."""
    import torch
    p = Ar.shape[0]
    Yr = torch.empty((p, p), dtype=torch.float64, device=Ar.device)
    Yi = torch.empty_like(Yr)
    pa, lda = _mat(Ar, p, p, "Ar"); pai, ldai = _mat(Ai, p, p, "Ai")
    pc, ldc = _mat(Cr, p, p, "Cr"); pci, ldci = _mat(Ci, p, p, "Ci")
    if lda != ldai or ldc != ldci:
        raise ValueError("planar pairs must share a leading dimension")
    h.bind_stream()
    o, r = _newton_opts(tol, max_iter, **inv), _lib.frob_newton_result_t()
    vp = ctypes.c_void_p
    _lib.check(_lib.load().frob_lyapunov(h.ptr, p, pa, pai, lda, pc, pci, ldc, vp(Yr.data_ptr()), vp(Yi.data_ptr()),
                                         p, ctypes.byref(o), ctypes.byref(r)), "frob_lyapunov", r.inv)
    return Yr, Yi, r.as_dict()


def frob_inv_tower(h: Handle, tau, C, *, shift=FROB_SHIFT_AUTO, mu=0.0, seed=0, refine=0, prec=FROB_PREC_F64):
    """Inverse of X = sum_alpha C[p] xi^alpha over the iterated quadratic extension
    with xi_k^2 = -tau[k] (Section 2.4).  C: list of 2^m float64 (n, n) device
    tensors (plane p = coefficient of xi^alpha, alpha_k = bit k of p).
    Returns (list of 2^m planes of X^{-1}, result dict)."""
    import torch
    m = len(tau)
    if len(C) != 1 << m:
        raise ValueError("C must hold 2^m planes")
    n = C[0].shape[0]
    lds = set()
    ptrs = []
    for p, t in enumerate(C):
        pt, ld = _mat(t, n, n, f"C[{p}]")
        ptrs.append(pt)
        lds.add(ld)
    if len(lds) != 1:
        raise ValueError("all planes must share a leading dimension")
    X = [torch.empty((n, n), dtype=torch.float64, device=C[0].device) for _ in C]
    h.bind_stream()
    vp = ctypes.c_void_p
    cin = (vp * len(C))(*[p.value for p in ptrs])
    xout = (vp * len(C))(*[x.data_ptr() for x in X])
    taus = (ctypes.c_double * m)(*[float(v) for v in tau])
    o, r = _opts(shift, mu, seed, refine, prec), frob_result_t()
    _lib.check(_lib.load().frob_inv_tower(h.ptr, m, n, taus, cin, lds.pop(), xout, n, ctypes.byref(o),
                                          ctypes.byref(r)), "frob_inv_tower", r)
    return X, r.as_dict()
