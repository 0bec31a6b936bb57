"""GPU parity of Frobenius inversion over iterated quadratic extensions
(Section 2.4, Theorem 2.10): F_m with xi_k^2 = -tau_k, against the oracle's
inverse from X Z = 1 through the real regular representation.  The Frobenius
route's error grows with the conditioning of the intermediate matrices
A + tau B A^{-1} B at every level; the bound used is 1e-9 relative
(Frobenius norm over all planes), and m = 1 reduces to complex inversion."""
import numpy as np
import pytest

import oracle
from _helpers import to_dev, to_host

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def h():
    import paper_2208_01239_amd as fi
    hd = fi.Handle(0)
    yield hd
    hd.close()


def rel(X, R):
    return float(np.sqrt(np.sum((X - R) ** 2) / np.sum(R ** 2)))


@pytest.mark.parametrize("tau,n", [((1.0,), 1), ((1.0,), 130), ((2.5,), 257), ((1.0,), 1100),
                                   ((1.0, 1.0), 3), ((1.0, 1.0), 200), ((2.0, 0.5), 513),
                                   ((1.0, 2.0, 0.5), 64), ((1.0, 1.0, 1.0), 150), ((3.0, 1.0, 1.0, 0.25), 40)])
def test_tower_inverse(h, tau, n):
    import paper_2208_01239_amd as fi
    m = len(tau)
    rng = np.random.default_rng(1000 * m + n)
    C = rng.standard_normal((1 << m, n, n))
    R, info = oracle.tower_inv(list(tau), C)
    assert info == 0
    X, res = fi.frob_inv_tower(h, list(tau), [to_dev(c) for c in C])
    Xh = np.stack([to_host(x) for x in X])
    e = rel(Xh, R)
    one = oracle.tower_mul(list(tau), C, Xh) if n <= 300 else None
    print(f"tower m={m} tau={tau} n={n}: relF {e:.2e}"
          + ("" if one is None else f", ||X X^-1 - 1||_max {np.abs(one - np.eye(n)[None] * (np.arange(1 << m) == 0)[:, None, None]).max():.1e}"))
    assert e <= 1e-9


def test_tower_bicomplex_split_on_gpu(h):
    """Bicomplex (m = 2, tau = (1, 1)) against two complex inverses through the
    idempotents (1 +- ij)/2, computed by the oracle's Algorithm 4."""
    import paper_2208_01239_amd as fi
    n = 90
    C = np.random.default_rng(5).standard_normal((4, n, n))
    X, _ = fi.frob_inv_tower(h, [1.0, 1.0], [to_dev(c) for c in C])
    Xh = np.stack([to_host(x) for x in X])
    W1r, W1i, _, _, _ = oracle.cinv_lu(C[0] + C[3], C[1] - C[2])    # Z1 - i Z2
    W2r, W2i, _, _, _ = oracle.cinv_lu(C[0] - C[3], C[1] + C[2])    # Z1 + i Z2
    ref = np.stack([(W1r + W2r) / 2, (W1i + W2i) / 2, -(W1i - W2i) / 2, (W1r - W2r) / 2])
    assert rel(Xh, ref) <= 1e-10


def test_tower_argument_checks(h):
    import paper_2208_01239_amd as fi
    C = [to_dev(np.eye(4)) for _ in range(2)]
    with pytest.raises(fi.FrobError):
        fi.frob_inv_tower(h, [-1.0], C)
    with pytest.raises(ValueError):
        fi.frob_inv_tower(h, [1.0, 1.0], C)
