"""GPU parity of the conditioning-aware variants of Frobenius inversion.

* FROB_SHIFT_PHASE inverts e^{i theta} M and rotates back.  theta = atan(mu)
  is Algorithm 6 (Section 4.2, up to the scaling 1 / sqrt(1 + mu^2) of the
  shifted matrix); theta = -pi/2 inverts B - iA and gives the alternative
  formula of Section 2.3 for invertible B,
      M^{-1} = B^{-1}A (A B^{-1} A + B)^{-1} - i (A B^{-1} A + B)^{-1}.
* kappa_1(C) = ||C||_1 ||C^{-1}||_1 is formed exactly from C and from the real
  part of the inverse (which is C^{-1}).
* FROB_SHIFT_COND tries theta = 0, -pi/2, pi/4, -pi/4 until u kappa_1(C) meets
  the target, keeping the best-conditioned inverse.
Every result is compared with the oracle's complex Gaussian elimination
(Algorithm 4)."""
import math

import numpy as np
import pytest

import oracle
from paper_2208_01239_amd import inputs
from _helpers import relF, to_dev, to_host

pytestmark = pytest.mark.gpu
U64 = 2.0 ** -53


@pytest.fixture(scope="module")
def h():
    import paper_2208_01239_amd as fi
    hd = fi.Handle(0)
    yield hd
    hd.close()


def _kC(A, B):
    return float(np.linalg.cond(A + B @ np.linalg.solve(A, B)))


@pytest.mark.parametrize("n,mu", [(40, 0.3), (300, 2.0), (1100, 0.7)])
def test_phase_rotation_is_algorithm6(h, n, mu):
    import paper_2208_01239_amd as fi
    A, B = inputs.general(n, 1200 + n)
    X1r, X1i, r1 = fi.frob_inv_general(h, to_dev(A), to_dev(B), shift=fi.FROB_SHIFT_PHASE, theta=math.atan(mu))
    X2r, X2i, r2 = fi.frob_inv_general(h, to_dev(A), to_dev(B), shift=fi.FROB_SHIFT_ON, mu=mu)
    Rr, Ri, _, _, _ = oracle.cinv_lu(A, B)
    Am, Bm = A - mu * B, mu * A + B
    tol = max(1e-10, 16 * U64 * _kC(Am, Bm))
    e1, e2 = relF(to_host(X1r), to_host(X1i), Rr, Ri), relF(to_host(X2r), to_host(X2i), Rr, Ri)
    print(f"phase n={n} theta=atan({mu}): relF {e1:.2e}; Algorithm 6 {e2:.2e}; tol {tol:.1e}")
    assert abs(r1["theta"] - math.atan(mu)) <= 1e-15
    assert e1 <= tol and e2 <= tol
    assert relF(to_host(X1r), to_host(X1i), to_host(X2r), to_host(X2i)) <= 2 * tol


@pytest.mark.parametrize("n", [5, 200, 1100])
def test_b_invertible_formula(h, n):
    """theta = -pi/2 with a singular real part (a zero column in A) and an
    invertible B: Algorithm 5 stops at stage 1, the B formula inverts M.  The
    result also matches the printed formula evaluated with LAPACK."""
    import paper_2208_01239_amd as fi
    A, B = inputs.general(n, 1300 + n)
    A[:, n // 2] = 0.0
    with pytest.raises(fi.FrobSingularError) as ex:
        fi.frob_inv_general(h, to_dev(A), to_dev(B), shift=fi.FROB_SHIFT_OFF)
    assert ex.value.result.stage == 1
    Xr, Xi, r = fi.frob_inv_general(h, to_dev(A), to_dev(B), shift=fi.FROB_SHIFT_PHASE, theta=-math.pi / 2)
    Rr, Ri, info, _, _ = oracle.cinv_lu(A, B)
    assert info == 0
    Cp = A @ np.linalg.solve(B, A) + B
    tol = max(1e-10, 16 * U64 * np.linalg.cond(Cp))
    e = relF(to_host(Xr), to_host(Xi), Rr, Ri)
    Ci = np.linalg.inv(Cp)
    Fr, Fi = np.linalg.solve(B, A) @ Ci, -Ci
    print(f"B formula n={n}: relF {e:.2e} (tol {tol:.1e}); vs printed formula {relF(to_host(Xr), to_host(Xi), Fr, Fi):.2e}")
    assert e <= tol
    assert relF(to_host(Xr), to_host(Xi), Fr, Fi) <= tol


@pytest.mark.parametrize("n", [64, 513])
def test_cond1_of_c_is_exact(h, n):
    import paper_2208_01239_amd as fi
    A, B = inputs.general(n, 1400 + n)
    _, _, r = fi.frob_inv_general(h, to_dev(A), to_dev(B), report_cond=True)
    C = A + B @ np.linalg.solve(A, B)
    ref = np.linalg.cond(C, 1)
    print(f"kappa_1(C) n={n}: {r['cond1_C']:.6e} vs numpy {ref:.6e}")
    assert abs(r["cond1_C"] - ref) <= 1e-6 * ref


def _hard_real_part(n, seed):
    """A = 1e-3 Q1 diag(1 .. 1e-6) Q2 (log-spaced, Haar orthogonal factors),
    B = I + H / (4 sqrt(n)): C = A + B A^{-1} B has kappa_1 ~ 1e7, while
    C' = B + A B^{-1} A is close to B and M = A + iB has kappa ~ 2."""
    rng = np.random.default_rng(seed)
    Q1, _ = np.linalg.qr(rng.standard_normal((n, n)))
    Q2, _ = np.linalg.qr(rng.standard_normal((n, n)))
    A = 1e-3 * (Q1 * np.logspace(0, -6, n)) @ Q2
    B = np.eye(n) + rng.standard_normal((n, n)) / (4 * np.sqrt(n))
    return A, B


@pytest.mark.parametrize("n", [100, 1100])
def test_cond_mode_picks_the_b_formula(h, n):
    import paper_2208_01239_amd as fi
    A, B = _hard_real_part(n, 1500 + n)
    Rr, Ri, info, _, _ = oracle.cinv_lu(A, B)
    assert info == 0
    P = fi.frob_inv_general(h, to_dev(A), to_dev(B), report_cond=True)
    X = fi.frob_inv_general(h, to_dev(A), to_dev(B), shift=fi.FROB_SHIFT_COND, cond_tol=1e-13)
    ep, ex_ = relF(to_host(P[0]), to_host(P[1]), Rr, Ri), relF(to_host(X[0]), to_host(X[1]), Rr, Ri)
    print(f"cond mode n={n}: plain kappa_1(C) {P[2]['cond1_C']:.2e} relF {ep:.2e}; chosen theta {X[2]['theta']:.3f} "
          f"kappa_1 {X[2]['cond1_C']:.2e} relF {ex_:.2e}, tried {X[2]['shifts_tried']}")
    assert abs(X[2]["theta"] + math.pi / 2) <= 1e-15 and X[2]["shifts_tried"] == 2
    assert X[2]["cond1_C"] < P[2]["cond1_C"] / 1e3
    assert ex_ <= 1e-12 and ep > 10 * ex_


def test_cond_mode_accepts_a_good_first_rotation(h):
    import paper_2208_01239_amd as fi
    A, B = inputs.hpd(200, 9)    # kappa(C) <= kappa(M) ~ 5: theta = 0 meets any sensible target
    X = fi.frob_inv_general(h, to_dev(A), to_dev(B), shift=fi.FROB_SHIFT_COND)
    Rr, Ri, _, _ = oracle.cinv_chol(A, B)
    assert X[2]["shifts_tried"] == 1 and X[2]["theta"] == 0.0
    assert relF(to_host(X[0]), to_host(X[1]), Rr, Ri) <= 1e-12
