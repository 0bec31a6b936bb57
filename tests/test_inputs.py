"""The seeded input generators: reproducibility across array backends and the
properties their constructions promise (no oracle arithmetic here)."""
import numpy as np
import pytest

from paper_2208_01239_amd import inputs


@pytest.mark.parametrize("kind", ["general", "hpd"])
@pytest.mark.parametrize("n", [1, 2, 7, 64, 257])
def test_rotation_spectrum_numpy_torch_bit_identical(kind, n):
    """The rotation-built spectrum input is assembled by the same elementwise
    IEEE operations in numpy and in torch: identical bits (here torch on the
    CPU; the GPU tests compare SHA-256 digests with the host's)."""
    import torch
    A, B = inputs.spectrum_rotations(n, 1e4, kind, seed=11)
    At, Bt = inputs.spectrum_rotations(n, 1e4, kind, seed=11, device="cpu")
    assert isinstance(At, torch.Tensor)
    assert np.array_equal(A.view(np.uint64), At.numpy().view(np.uint64))
    assert np.array_equal(B.view(np.uint64), Bt.numpy().view(np.uint64))


@pytest.mark.parametrize("kind", ["general", "hpd"])
@pytest.mark.parametrize("n,kappa", [(64, 1e2), (200, 1e6), (255, 1e4)])
def test_rotation_spectrum_singular_values(kind, n, kappa):
    """Singular values are sigma_j = kappa^(-j/(n-1)) up to rounding; the HPD
    form is exactly Hermitian with positive eigenvalues (then A = Re M is
    symmetric positive definite and B = Im M skew, Lemma 4.5)."""
    A, B = inputs.spectrum_rotations(n, kappa, kind, seed=3)
    M = A + 1j * B
    s = np.linalg.svd(M, compute_uv=False)
    sig = kappa ** (-np.arange(n) / (n - 1))
    assert np.allclose(s, sig, rtol=1e-13, atol=1e-15)
    if kind == "hpd":
        assert np.array_equal(A, A.T) and np.array_equal(B, -B.T)
        w = np.linalg.eigvalsh(M)
        assert w.min() > 0.5 / kappa
        np.linalg.cholesky(A)
    else:
        # generic: the real part is not Hermitian-structured
        assert not np.allclose(A, A.T)


def test_rotation_levels_unitary_and_dense():
    """Each pair rotation is unitary to rounding, and the assembled unitary
    has no structural zeros at n = 128 (the levels mix every row)."""
    rng = np.random.default_rng(0)
    for perm, ar, ai, br, bi in inputs._rotation_levels(128, rng):
        assert sorted(perm) == list(range(128))
        assert np.abs(ar * ar + ai * ai + br * br + bi * bi - 1.0).max() <= 8 * 2.0 ** -53
    A, B = inputs.spectrum_rotations(128, 1.0, "general", seed=0)
    assert np.all(np.abs(A) + np.abs(B) > 0)
    M = A + 1j * B
    assert np.abs(M @ M.conj().T - np.eye(128)).max() <= 1e-13   # kappa = 1: M itself is unitary
