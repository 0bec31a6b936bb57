"""GPU parity of the mixed-precision path: FP32 / BF16 matrix-core products in
the factorizations, then Newton-Schulz refinement with the residual I - M X
formed in FP64.  Inputs are the spectrum-controlled matrices
M = U diag(sigma) V^H (sigma log-spaced, kappa(M) = kappa; V = U for HPD) at a
size the oracle finishes in a second; references are the oracle's complex
Gaussian elimination (Algorithm 4) and complex Cholesky inversion (Algorithm 8).
"""
import math

import numpy as np
import pytest

import oracle
from paper_2208_01239_amd import inputs
from _helpers import relF, to_dev, to_host

pytestmark = pytest.mark.gpu

TOL = 1e-10
N = 384


@pytest.fixture(scope="module")
def h():
    import paper_2208_01239_amd as fi
    hd = fi.Handle(0)
    yield hd
    hd.close()


def _case(kind, kappa):
    seed = (300 if kind == "general" else 400) + int(round(math.log10(kappa)))
    A, B = inputs.spectrum(N, kappa, kind, seed=seed)
    ref = oracle.cinv_lu(A, B) if kind == "general" else oracle.cinv_chol(A, B)
    return A, B, ref[0], ref[1]


def _inv(h, kind, A, B, **kw):
    import paper_2208_01239_amd as fi
    f = fi.frob_inv_general if kind == "general" else fi.frob_inv_hpd
    Xr, Xi, res = f(h, to_dev(A), to_dev(B), **kw)
    return to_host(Xr), to_host(Xi), res


@pytest.mark.parametrize("kind,prec,kappa", [
    ("general", 1, 1e2), ("general", 1, 1e4),
    ("hpd", 1, 1e2), ("hpd", 1, 1e4), ("hpd", 1, 1e6),
    ("hpd", 2, 1e2),
])
def test_mixed_precision_refined_to_fp64(h, kind, prec, kappa):
    A, B, Rr, Ri = _case(kind, kappa)
    X0r, X0i, _ = _inv(h, kind, A, B, prec=prec)
    e0 = relF(X0r, X0i, Rr, Ri)
    Xr, Xi, res = _inv(h, kind, A, B, prec=prec, refine=8)
    e = relF(Xr, Xi, Rr, Ri)
    print(f"{kind} prec {prec} kappa {kappa:.0e}: unrefined {e0:.2e} -> refined {e:.2e} in "
          f"{res['refine_steps']} steps; ||I-MX||/sqrt(n) {res['resid0']:.2e} -> {res['resid']:.2e}")
    # the low-precision operands really were used ...
    assert e0 > 1e-9
    # ... and refinement recovers the FP64 bar
    assert e <= TOL
    assert res["refine_steps"] >= 1 and res["resid"] < res["resid0"]


@pytest.mark.parametrize("kappa", [1e2, 1e4, 1e6])
def test_f32_correction_after_fp64_factorization(h, kappa):
    """FP64 factorizations, FP64 residual, FP32 correction X R: the correction
    is as small as the error of X, so its FP32 rounding costs only a factor of
    about u_32 kappa(M) per step, against (I - M X)^2 for the FP64 step."""
    A, B, Rr, Ri = _case("general", kappa)
    X0r, X0i, _ = _inv(h, "general", A, B)
    e0 = relF(X0r, X0i, Rr, Ri)
    X1r, X1i, r64 = _inv(h, "general", A, B, refine=1, refine_tol=1e-300)
    e64 = relF(X1r, X1i, Rr, Ri)
    X2r, X2i, r32 = _inv(h, "general", A, B, refine=1, refine_tol=1e-300, f32_correction=True)
    e32 = relF(X2r, X2i, Rr, Ri)
    X8r, X8i, r8 = _inv(h, "general", A, B, refine=8, f32_correction=True)
    e8 = relF(X8r, X8i, Rr, Ri)
    print(f"kappa {kappa:.0e}: unrefined {e0:.2e}, one FP64 step {e64:.2e}, one FP32-correction step {e32:.2e}, "
          f"{r8['refine_steps']} FP32-correction steps {e8:.2e}")
    # the same FP64 factorizations and residual before the first step
    assert abs(r32["resid0"] - r64["resid0"]) <= 1e-12 * r64["resid0"]
    assert r32["refine_steps"] == 1
    # the flag is honoured: the correction was rounded differently
    assert not np.array_equal(X1r, X2r)
    # one step gains at least u_32 kappa(M) (6e-8 kappa), with a margin of 20
    assert e32 <= max(20 * 6e-8 * kappa * e0, 10 * e64, 1e-13)
    assert e8 <= TOL and r8["resid"] < r8["resid0"]


def test_newton_schulz_squares_the_residual(h):
    """I - M X_{k+1} = (I - M X_k)^2, so ||R_1||_F <= ||R_0||_F^2 (up to FP64 rounding)."""
    A, B, Rr, Ri = _case("general", 1e2)
    _, _, res = _inv(h, "general", A, B, prec=1, refine=1, refine_tol=1e-300)
    f0 = res["resid0"] * math.sqrt(N)
    f1 = res["resid"] * math.sqrt(N)
    print(f"||R0||_F {f0:.3e}  ||R1||_F {f1:.3e}  ||R0||_F^2 {f0 * f0:.3e}")
    assert res["refine_steps"] == 1
    assert f1 <= 1.01 * f0 * f0 + 1e-10


def test_no_convergence_reported(h):
    """BF16 operands on a general matrix with kappa = 1e4: ||I - M X0||_F >= 1, so
    the start needs the spectral-norm estimate.  Either refinement is refused
    (estimate >= 1, or the residual grew and X0 was restored) -- then X is the
    unrefined inverse, bit for bit -- or it converges to the FP64 bar."""
    import paper_2208_01239_amd as fi
    import torch
    A, B, Rr, Ri = _case("general", 1e4)
    dA, dB = to_dev(A), to_dev(B)
    U = fi.frob_inv_general(h, dA, dB, prec=2)
    Xr, Xi = torch.empty_like(dA), torch.empty_like(dA)
    try:
        _, _, res = fi.frob_inv_general(h, dA, dB, Xr, Xi, prec=2, refine=8)
    except fi.FrobNoConvergenceError as ex:
        r = ex.result
        print(f"bf16 general: refused, resid0 {r.resid0:.2e}, norm2_est {r.norm2_est:.2e}")
        assert r.refine_steps == 0 and r.resid0 * math.sqrt(N) >= 1.0 and r.norm2_est > 0.0
        assert torch.equal(Xr, U[0]) and torch.equal(Xi, U[1])
        return
    print(f"bf16 general: converged in {res['refine_steps']} steps, norm2_est {res['norm2_est']:.2e}")
    assert relF(to_host(Xr), to_host(Xi), Rr, Ri) <= TOL


def test_fp64_precision_flag_is_default(h):
    A, B, Rr, Ri = _case("general", 1e2)
    Xr, Xi, _ = _inv(h, "general", A, B)
    Yr, Yi, _ = _inv(h, "general", A, B, prec=0)
    assert np.array_equal(Xr, Yr) and np.array_equal(Xi, Yi)
    assert relF(Xr, Xi, Rr, Ri) <= TOL
