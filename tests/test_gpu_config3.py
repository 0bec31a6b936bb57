"""Mixed precision at n = 8192 against the FP64 oracle.

Inputs: M = U diag(sigma) W (general) and U diag(sigma) U^H (HPD) with
sigma log-spaced to kappa in {1e2, 1e4, 1e6}, U and W built from random pair
rotations and row permutations (``inputs.spectrum_rotations``, seeds
300 + log10 kappa and 400 + log10 kappa).  The device rebuilds the matrix
with torch from the same host-drawn coefficients; its SHA-256 must equal the
one stored beside the oracle samples before any value is compared.

The oracle samples (one column per 64-column band, 256 seeded rows) come from
complex GEPP plus refinement with double-double residuals, accurate to about
u even at kappa = 1e6, so the errors below are the path's own.

Every result of the refined paths (FP64, FP32 and BF16 matrix-core operands,
Newton-Schulz with the residual in FP64) must either meet

    relF <= max(1e-10, 32 u kappa(M))

(after refinement the forward error is bounded by the residual, and an FP64
residual of M X cannot be smaller than about u kappa(M)), or be refused with a
status that names why: FROB_NO_CONVERGENCE, which the refinement returns only
from a start with ||I - M X_0||_F >= 1 whose 2-norm estimate is >= 1 or whose
residual then grew (Newton-Schulz cannot contract from there), or, for
BF16 operands on HPD input, FROB_NOT_HPD when the BF16-rounded Cholesky
breaks down.  FP64 and FP32 on the HPD inputs are required to converge."""
import hashlib
import os

import numpy as np
import pytest

from paper_2208_01239_amd import inputs
from _helpers import relF

pytestmark = pytest.mark.gpu
TOL = 1e-10
U64 = 2.0 ** -53
N = 8192
HERE = os.path.dirname(os.path.abspath(__file__))


@pytest.fixture(scope="module")
def h():
    import paper_2208_01239_amd as fi
    hd = fi.Handle(0)
    yield hd
    hd.close()


def _sha_dev(t):
    return hashlib.sha256(t.cpu().numpy().tobytes()).hexdigest()


@pytest.mark.parametrize("kind", ["general", "hpd"])
@pytest.mark.parametrize("kexp", [2, 4, 6])
def test_config3_against_oracle(h, kind, kexp):
    import paper_2208_01239_amd as fi
    import torch
    path = os.path.join(HERE, "golden", f"n{N}_rot_{kind}_k1e{kexp}_band_samples.npz")
    if not os.path.exists(path):
        pytest.skip("oracle samples not generated")
    g = np.load(path, allow_pickle=False)
    kappa = 10.0 ** kexp
    seed = (300 if kind == "general" else 400) + kexp
    dA, dB = inputs.spectrum_rotations(N, kappa, kind, seed=seed, device="cuda")
    assert _sha_dev(dA) == str(g["sha_a"]) and _sha_dev(dB) == str(g["sha_b"]), \
        "device-built input is not bit-identical to the oracle's"
    rows = torch.from_numpy(g["rows"]).cuda()
    cols = torch.from_numpy(g["cols"]).cuda()
    Xr, Xi = torch.empty_like(dA), torch.empty_like(dA)
    fn = fi.frob_inv_general if kind == "general" else fi.frob_inv_hpd

    def err():
        xr = Xr.index_select(0, rows).index_select(1, cols).cpu().numpy()
        xi = Xi.index_select(0, rows).index_select(1, cols).cpu().numpy()
        return relF(xr, xi, g["xr"], g["xi"])

    tol = max(TOL, 32 * U64 * kappa)
    lines = []
    for pname, prec in (("f64", fi.FROB_PREC_F64), ("f32", fi.FROB_PREC_F32), ("bf16", fi.FROB_PREC_BF16)):
        try:
            fn(h, dA, dB, Xr, Xi, prec=prec)
            e0 = err()
        except fi.FrobNotHPDError as ex:
            assert kind == "hpd" and prec == fi.FROB_PREC_BF16, ex
            lines.append(f"{pname}: BF16 Cholesky breakdown (stage {ex.result.stage}, info {ex.result.info})")
            continue
        try:
            _, _, res = fn(h, dA, dB, Xr, Xi, prec=prec, refine=8)
            e1 = err()
            lines.append(f"{pname}: unrefined {e0:.2e}, refined {e1:.2e} in {res['refine_steps']} steps "
                         f"(||R0||_2 est {res['norm2_est']:.2e})")
            assert e1 <= tol, (pname, e1, tol)
        except fi.FrobNoConvergenceError as ex:
            lines.append(f"{pname}: unrefined {e0:.2e}, refused: ||R0||_2 est {ex.result.norm2_est:.2e}")
            assert not (kind == "hpd" and prec != fi.FROB_PREC_BF16), ex
            assert ex.result.resid0 * np.sqrt(N) >= 1.0, ex
    print(f"n={N} {kind} kappa=1e{kexp} (tol {tol:.1e}): " + "; ".join(lines))
    del dA, dB, Xr, Xi
    torch.cuda.empty_cache()
