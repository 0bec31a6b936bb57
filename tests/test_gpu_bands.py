"""Large-order parity on one sampled column in every 64-column band.

The stored values (tests/golden/*_band_samples.npz, written by
make_band_samples.py from the oracle alone) are entries X[rows, cols] of the
inverse with one column in each 64-column band, so every panel of the blocked
LU and Cholesky factorizations, and every band of the carried columns, owns
at least one checked column; 256 seeded rows are kept of each column.  Each
file holds the SHA-256 of the input the oracle saw; inputs that are exact
draws (iid Gaussian) must match it bit for bit, so the comparison is never
made against a different matrix.

Tolerances: the FP64 Frobenius result without refinement is held to
16 u kappa_2(C) (C = A + B A^{-1} B, from the stored metadata at n = 4096) or
to 1e-7 at n = 8192 (no condition number stored there); the refined result
and both complex baselines to the 1e-10 bar."""
import hashlib
import os

import numpy as np
import pytest

from paper_2208_01239_amd import inputs
from _helpers import relF, to_dev

pytestmark = pytest.mark.gpu
TOL = 1e-10
U64 = 2.0 ** -53
HERE = os.path.dirname(os.path.abspath(__file__))


def _golden(name):
    path = os.path.join(HERE, "golden", name)
    if not os.path.exists(path):
        pytest.skip(f"{name} not generated")
    return np.load(path, allow_pickle=False)


def _sha(a):
    return hashlib.sha256(np.ascontiguousarray(a, dtype=np.float64).tobytes()).hexdigest()


@pytest.fixture(scope="module")
def h():
    import paper_2208_01239_amd as fi
    hd = fi.Handle(0)
    yield hd
    hd.close()


def _err(Xr, Xi, g):
    import torch
    r = torch.from_numpy(g["rows"]).to(Xr.device)
    c = torch.from_numpy(g["cols"]).to(Xr.device)
    xr = Xr.index_select(0, r).index_select(1, c).cpu().numpy()
    xi = Xi.index_select(0, r).index_select(1, c).cpu().numpy()
    return relF(xr, xi, g["xr"], g["xi"])


def _bands_covered(g, n):
    cols = g["cols"]
    assert np.array_equal(cols // 64, np.arange((n + 63) // 64)), "one sampled column per 64-column band"


@pytest.mark.parametrize("n", [4096, 8192])
def test_general_band_samples(h, n):
    import paper_2208_01239_amd as fi
    import torch
    g = _golden(f"n{n}_general_band_samples.npz")
    _bands_covered(g, n)
    A, B = inputs.general(n, 0)
    assert _sha(A) == str(g["sha_a"]) and _sha(B) == str(g["sha_b"]), "input differs from the oracle's"
    dA, dB = to_dev(A), to_dev(B)
    del A, B
    Xr, Xi = torch.empty_like(dA), torch.empty_like(dA)
    fi.frob_inv_general(h, dA, dB, Xr, Xi)
    e0 = _err(Xr, Xi, g)
    fi.frob_inv_general(h, dA, dB, Xr, Xi, refine=1, f32_correction=True, final_resid=False)
    e1 = _err(Xr, Xi, g)
    ez = []
    for form in (1, 0):
        fi.frob_cinv_lu(h, dA, dB, Xr, Xi, form=form)
        ez.append(_err(Xr, Xi, g))
    if n == 4096:
        meta = _golden("n4096_general_samples.npz")
        tol0 = 16 * U64 * float(meta["kappa_C"])
    else:
        tol0 = 1e-7
    print(f"n={n} general, {g['cols'].size} bands: plain {e0:.2e} (tol {tol0:.1e}), refined {e1:.2e}, "
          f"complex LU forms 1/0 {ez[0]:.2e}/{ez[1]:.2e}; oracle final correction {float(g['last_correction']):.1e}")
    assert e0 <= tol0
    assert e1 <= TOL
    assert max(ez) <= TOL
    del dA, dB, Xr, Xi
    torch.cuda.empty_cache()


def test_hpd_band_samples_n4096(h):
    import paper_2208_01239_amd as fi
    import torch
    g = _golden("n4096_hpd_band_samples.npz")
    _bands_covered(g, 4096)
    A, B = inputs.hpd(4096, 1)
    same = _sha(A) == str(g["sha_a"]) and _sha(B) == str(g["sha_b"])
    # Z Z^H is a BLAS product: another host may round it differently.  kappa(M)
    # is about 3 here, so a perturbation of a few units of roundoff in M moves
    # the inverse by far less than the 1e-10 bar; the comparison stands either way.
    dA, dB = to_dev(A), to_dev(B)
    Xr, Xi, _ = fi.frob_inv_hpd(h, dA, dB)
    e = _err(Xr, Xi, g)
    ec = []
    for form in (0, 1):
        fi.frob_cinv_chol(h, dA, dB, Xr, Xi, form=form)
        ec.append(_err(Xr, Xi, g))
    print(f"n=4096 hpd, 64 bands: frobenius {e:.2e}, complex Cholesky forms 0/1 {ec[0]:.2e}/{ec[1]:.2e}; "
          f"input bit-identical to the oracle's: {same}")
    assert e <= TOL and max(ec) <= TOL
    del dA, dB, Xr, Xi
    torch.cuda.empty_cache()
