"""Seeded synthetic inputs shared by the tests, the benchmark and the oracle runs.

This module only draws random numbers and assembles test matrices; it holds
none of the inversion arithmetic.  Every generator is deterministic in its seed
(numpy ``default_rng``, PCG64).  Shapes and distributions follow the workloads
of the paper (Section 5) and the synthetic configurations used for measurement:

* ``general``      -- A, B iid N(0, 1) (A invertible with probability 1).
* ``hpd``          -- M = Z Z^H + n I with Z complex, N(0, 1/2) per part;
                      A = Re M (SPD), B = Im M (skew), Lemma 4.5.
* ``paper_accuracy`` -- A = Q Lambda Q^T / ||Lambda||_F with kappa(A) = kappa
                      (Section 5.1 accuracy experiment), same for B.
* ``paper_speed``  -- A, B ~ U[0, 1] (Section 5.1 speed experiment).
* ``paper_hpd_speed`` -- (A + iB)^H (A + iB) + 0.01 I, A, B ~ U[-1, 1]
                      (Section 5.6).
* ``ill_conditioned_pair`` -- the construction in the proof of Theorem 3.5:
                      A = Q R, B = Q N R with N a direct sum of 2x2 blocks
                      [[0, -t], [t, 0]].
* ``spectrum``     -- M = U diag(sigma) V^H (or U diag(sigma) U^H) with Haar
                      U, V and sigma log-spaced to a target condition number.
* ``spectrum_device`` -- the same recipe at large orders, drawn and assembled
                      with torch on a device (its own random stream), with
                      the inverse V diag(1/sigma) U^H from the same factors.
* ``spectrum_rotations`` -- M = U diag(sigma) W (HPD: U diag(sigma) U^H)
                      with U, W products of random 2 x 2 unitary rotations
                      between random row permutations, built from row
                      operations alone, so that numpy on a host and torch on
                      a device produce the same bits (the input of the
                      mixed-precision workloads at large order).
* ``batch``        -- uneven batch: n ~ U{16..512}, kinds alternate general/HPD.
* ``spd_pair``     -- A = G1 G1^T / n + I and B = G2 G2^T / n + I with G1, G2
                      iid N(0, 1): both symmetric positive definite (the class
                      closing Section 4.3).
* ``sign_problem`` -- X = Z J Z^{-1} with Z uniform in [-1, 1] (both parts)
                      and J diagonal, half the eigenvalues with positive and
                      half with negative real part, away from zero (Section
                      5.3), with sign(X) = Z diag(+-1) Z^{-1} beside it.
* ``sylvester_problem`` -- A = Z J Z^{-1} with Re J in [9, 10] (sign(A) = I),
                      B likewise or B = A^H (Lyapunov), Y uniform in [-1, 1],
                      C = A Y + Y B (Section 5.4).
* ``polar_problem`` -- X = U P with U the unitary factor of a QR of a uniform
                      complex matrix and P = Z^H Z (Section 5.5).
"""
from __future__ import annotations

import numpy as np


def general(n: int, seed: int = 0):
    rng = np.random.default_rng(seed)
    A = rng.standard_normal((n, n))
    B = rng.standard_normal((n, n))
    return A, B


def hpd(n: int, seed: int = 1):
    rng = np.random.default_rng(seed)
    Zr = rng.standard_normal((n, n)) * np.sqrt(0.5)
    Zi = rng.standard_normal((n, n)) * np.sqrt(0.5)
    # Z Z^H with Z = Zr + i Zi, real and imaginary parts assembled from real products
    Mr = Zr @ Zr.T + Zi @ Zi.T
    Mi = Zi @ Zr.T - Zr @ Zi.T
    Mr = 0.5 * (Mr + Mr.T) + n * np.eye(n)
    Mi = 0.5 * (Mi - Mi.T)
    return np.ascontiguousarray(Mr), np.ascontiguousarray(Mi)


def _haar_orthogonal(n: int, rng) -> np.ndarray:
    Q, R = np.linalg.qr(rng.uniform(-1.0, 1.0, size=(n, n)))
    return Q * np.sign(np.diag(R))


def paper_accuracy(n: int, kappa: float = 10.0, seed: int = 2):
    rng = np.random.default_rng(seed)

    def one():
        Q = _haar_orthogonal(n, rng)
        if n == 1:
            lam = np.array([rng.choice([-1.0, 1.0])])
        else:
            mags = np.concatenate([[kappa], rng.uniform(1.0, kappa, size=n - 2), [1.0]])
            lam = mags * rng.choice([-1.0, 1.0], size=n)
        X = (Q * lam) @ Q.T / np.linalg.norm(lam)
        return 0.5 * (X + X.T)

    return one(), one()


def paper_speed(n: int, seed: int = 3):
    rng = np.random.default_rng(seed)
    return rng.uniform(0.0, 1.0, size=(n, n)), rng.uniform(0.0, 1.0, size=(n, n))


def paper_hpd_speed(n: int, seed: int = 6):
    rng = np.random.default_rng(seed)
    Ar = rng.uniform(-1.0, 1.0, size=(n, n))
    Ai = rng.uniform(-1.0, 1.0, size=(n, n))
    # (Ar + i Ai)^H (Ar + i Ai) = (Ar^T Ar + Ai^T Ai) + i (Ar^T Ai - Ai^T Ar)
    Mr = Ar.T @ Ar + Ai.T @ Ai + 0.01 * np.eye(n)
    Mi = Ar.T @ Ai - Ai.T @ Ar
    return np.ascontiguousarray(0.5 * (Mr + Mr.T)), np.ascontiguousarray(0.5 * (Mi - Mi.T))


def ill_conditioned_pair(m: int, t: float, seed: int = 7, identity_a: bool = False):
    """Theorem 3.5 construction on 2m x 2m matrices.  Returns (A, B, Q, R, N)."""
    n = 2 * m
    rng = np.random.default_rng(seed)
    if identity_a:
        Q = np.eye(n)
        R = np.eye(n)
    else:
        Q, R = np.linalg.qr(rng.standard_normal((n, n)))
    N = np.zeros((n, n))
    for b in range(m):
        N[2 * b, 2 * b + 1] = -t
        N[2 * b + 1, 2 * b] = t
    A = Q @ R
    B = Q @ N @ R
    return A, B, Q, R, N


def haar_unitary(n: int, rng):
    G = (rng.standard_normal((n, n)) + 1j * rng.standard_normal((n, n))) / np.sqrt(2.0)
    Q, R = np.linalg.qr(G)
    d = np.diag(R)
    return Q * (d / np.abs(d))


def spectrum(n: int, kappa: float, kind: str = "general", seed: int = 302):
    """M = U diag(sigma) V^H with sigma_j = kappa^(-j/(n-1)); HPD uses V = U."""
    rng = np.random.default_rng(seed)
    U = haar_unitary(n, rng)
    sig = kappa ** (-np.arange(n) / max(n - 1, 1))
    if kind == "hpd":
        M = (U * sig) @ U.conj().T
        M = 0.5 * (M + M.conj().T)
    else:
        V = haar_unitary(n, rng)
        M = (U * sig) @ V.conj().T
    return np.ascontiguousarray(M.real), np.ascontiguousarray(M.imag)


def spectrum_device(n: int, kappa: float, kind: str = "general", seed: int = 302, device: str = "cuda"):
    """Large-order form of ``spectrum``: U, V Haar (QR of complex Gaussians
    with the diagonal phases of R taken out), sigma_j = kappa^(-j/(n-1)),
    drawn with a seeded torch generator on ``device`` and assembled there in
    FP64.  Returns torch tensors (A, B, Re Minv, Im Minv) where
    Minv = V diag(1/sigma) U^H is built from the same factors (it is the
    inverse of the stored M to about u * kappa, relative)."""
    import torch

    g = torch.Generator(device=device)
    g.manual_seed(seed)

    def haar():
        re = torch.randn(n, n, generator=g, device=device, dtype=torch.float64)
        im = torch.randn(n, n, generator=g, device=device, dtype=torch.float64)
        Q, R = torch.linalg.qr(torch.complex(re, im) / np.sqrt(2.0))
        d = torch.diagonal(R)
        return Q * (d / d.abs())

    U = haar()
    V = U if kind == "hpd" else haar()
    sig = kappa ** (-torch.arange(n, device=device, dtype=torch.float64) / max(n - 1, 1))
    Vh = V.conj().T.contiguous()
    Uh = U.conj().T.contiguous()
    M = (U * sig) @ Vh
    Minv = (V * (1.0 / sig)) @ Uh
    if kind == "hpd":
        M = 0.5 * (M + M.conj().T)
        Minv = 0.5 * (Minv + Minv.conj().T)
    return (M.real.contiguous(), M.imag.contiguous(), Minv.real.contiguous(), Minv.imag.contiguous())


def _rotation_levels(n: int, rng):
    """Random levels of a unitary built from row operations: for each level a
    row permutation and, for the row pairs (2m, 2m + 1) of the permuted
    matrix, a 2 x 2 unitary [[alpha, beta], [-conj(beta), conj(alpha)]] with
    alpha = c e^{ia}, beta = s e^{ib}.  Cosine, sine and the phases come from
    the rational parametrisation ((1 - t^2), 2t) / (1 + t^2), so every
    coefficient is a few correctly rounded operations on uniform draws and
    the same on every machine."""
    h = n // 2
    levels = []
    for _ in range(2 * max(1, int(np.ceil(np.log2(max(n, 2)))))):
        perm = rng.permutation(n)
        t, pa, pb = rng.uniform(-1.0, 1.0, (3, h))
        sa, sb = (2.0 * rng.integers(0, 2, (2, h)) - 1.0)
        den = 1.0 + t * t
        c, s = (1.0 - t * t) / den, (2.0 * t) / den
        da, db = 1.0 + pa * pa, 1.0 + pb * pb
        ar, ai = c * (sa * ((1.0 - pa * pa) / da)), c * (sa * ((2.0 * pa) / da))
        br, bi = s * (sb * ((1.0 - pb * pb) / db)), s * (sb * ((2.0 * pb) / db))
        levels.append((perm, ar, ai, br, bi))
    return levels


def _mix_pairs(Xr, Xi, p, q, r, s):
    """Rows (2m, 2m + 1) -> (p a + q b, r a + s b) with complex coefficient
    vectors p, q, r, s given as (re, im) column vectors; plain products and
    sums in a fixed order (no fused multiply-add)."""
    h = Xr.shape[0] // 2
    ar, ai = Xr[0:2 * h:2], Xi[0:2 * h:2]
    br, bi = Xr[1:2 * h:2], Xi[1:2 * h:2]
    nar = p[0] * ar - p[1] * ai + q[0] * br - q[1] * bi
    nai = p[0] * ai + p[1] * ar + q[0] * bi + q[1] * br
    nbr = r[0] * ar - r[1] * ai + s[0] * br - s[1] * bi
    nbi = r[0] * ai + r[1] * ar + s[0] * bi + s[1] * br
    Xr[0:2 * h:2], Xi[0:2 * h:2] = nar, nai
    Xr[1:2 * h:2], Xi[1:2 * h:2] = nbr, nbi


def _apply_unitary(Xr, Xi, levels, adjoint, to):
    """X <- U X (adjoint: U^H X) for U = B_L P_L ... B_1 P_1, where P_k takes
    row perm_k[i] to row i and B_k is the level's pair rotation."""
    if not adjoint:
        for perm, ar, ai, br, bi in levels:
            idx = to(perm)
            Xr, Xi = Xr[idx], Xi[idx]
            a, b = (to(ar), to(ai)), (to(br), to(bi))
            _mix_pairs(Xr, Xi, a, b, (-b[0], b[1]), (a[0], -a[1]))
    else:
        # U^H = P_1^T B_1^H ... P_L^T B_L^H, B^H = [[conj(alpha), -beta], [conj(beta), alpha]]
        for perm, ar, ai, br, bi in reversed(levels):
            a, b = (to(ar), to(ai)), (to(br), to(bi))
            _mix_pairs(Xr, Xi, (a[0], -a[1]), (-b[0], -b[1]), (b[0], -b[1]), a)
            idx = to(np.argsort(perm))
            Xr, Xi = Xr[idx], Xi[idx]
    return Xr, Xi


def spectrum_rotations(n: int, kappa: float, kind: str = "general", seed: int = 302, device=None):
    """M = U diag(sigma) W (general) or U diag(sigma) U^H made exactly
    Hermitian (HPD), sigma_j = kappa^(-j/(n-1)), U and W random unitaries of
    2 ceil(log2 n) levels each (``_rotation_levels``).  All random draws and
    coefficients are made on the host with numpy; the matrix is assembled by
    row permutations, pair rotations and row scalings only, elementwise IEEE
    products and sums evaluated in one fixed order, either with numpy
    (device None: numpy arrays) or with torch on ``device`` (torch tensors).
    The two produce identical bits, so expected values computed on a host
    for the numpy matrix apply to the device matrix.  The singular values of
    M are sigma up to rounding (a few units of roundoff per level)."""
    rng = np.random.default_rng(seed)
    U = _rotation_levels(n, rng)
    W = U if kind == "hpd" else _rotation_levels(n, rng)
    # kappa ** x through the C library's pow on Python floats, not a vectorised power
    sig = np.array([float(kappa) ** (-(j / max(n - 1, 1))) for j in range(n)])
    if device is None:
        def to(a):
            return a[:, None] if a.ndim == 1 and a.dtype == np.float64 else a
        Xr, Xi = np.eye(n), np.zeros((n, n))
    else:
        import torch

        def to(a):
            t = torch.from_numpy(np.ascontiguousarray(a)).to(device)
            return t[:, None] if a.ndim == 1 and a.dtype == np.float64 else t
        Xr = torch.eye(n, dtype=torch.float64, device=device)
        Xi = torch.zeros((n, n), dtype=torch.float64, device=device)
    Xr, Xi = _apply_unitary(Xr, Xi, W, kind == "hpd", to)
    s = to(sig)
    Xr, Xi = Xr * s, Xi * s
    Xr, Xi = _apply_unitary(Xr, Xi, U, False, to)
    if kind == "hpd":
        Xr, Xi = 0.5 * (Xr + Xr.T), 0.5 * (Xi - Xi.T)
    if device is None:
        return np.ascontiguousarray(Xr), np.ascontiguousarray(Xi)
    return Xr.contiguous(), Xi.contiguous()


def batch(count: int = 2048, seed: int = 4, n_lo: int = 16, n_hi: int = 512):
    """Uneven batch: sizes n ~ U{n_lo..n_hi}; kind_i = i mod 2 (0 general, 1 HPD).
    Returns (ns, kinds, list of (A, B))."""
    rng = np.random.default_rng(seed)
    ns = rng.integers(n_lo, n_hi + 1, size=count)
    kinds = np.arange(count) % 2
    children = np.random.SeedSequence(seed).spawn(count)
    mats = []
    for i in range(count):
        s = int(children[i].generate_state(1)[0])
        n = int(ns[i])
        mats.append(general(n, s) if kinds[i] == 0 else hpd(n, s))
    return ns.astype(np.int32), kinds.astype(np.int32), mats


def adjoint_batch(count: int = 256, n: int = 256, seed: int = 5):
    """HPD matrices and complex weights W for L = sum_b Re tr(W_b X_b)."""
    children = np.random.SeedSequence(seed).spawn(2 * count)
    mats, ws = [], []
    for b in range(count):
        mats.append(hpd(n, int(children[b].generate_state(1)[0])))
        rng = np.random.default_rng(int(children[count + b].generate_state(1)[0]))
        ws.append((rng.standard_normal((n, n)), rng.standard_normal((n, n))))
    return mats, ws


def _uniform_complex(rng, shape):
    return rng.uniform(-1.0, 1.0, size=shape) + 1j * rng.uniform(-1.0, 1.0, size=shape)


def sign_problem(n: int, seed: int = 50):
    """(Xr, Xi, Sr, Si): X = Z J Z^{-1} and its sign Z diag(sign Re J) Z^{-1}."""
    rng = np.random.default_rng(seed)
    Z = _uniform_complex(rng, (n, n))
    re = rng.uniform(0.5, 2.0, n)
    re[n // 2:] *= -1.0
    J = re + 1j * rng.uniform(-1.0, 1.0, n)
    Zi = np.linalg.inv(Z)
    X = (Z * J) @ Zi
    S = (Z * np.sign(J.real)) @ Zi
    return (np.ascontiguousarray(X.real), np.ascontiguousarray(X.imag), np.ascontiguousarray(S.real),
            np.ascontiguousarray(S.imag))


def sylvester_problem(p: int, q: int, seed: int = 51, lyapunov: bool = False):
    """(A, B, C, Y) as complex numpy arrays with A Y + Y B = C, sign(A) = sign(B) = I."""
    rng = np.random.default_rng(seed)

    def stable(m):
        Z = _uniform_complex(rng, (m, m))
        J = rng.uniform(9.0, 10.0, m) + 1j * rng.uniform(-1.0, 1.0, m)
        return (Z * J) @ np.linalg.inv(Z)
    A = stable(p)
    B = A.conj().T.copy() if lyapunov else stable(q)
    Y = _uniform_complex(rng, (p, q if not lyapunov else p))
    C = A @ Y + Y @ B
    return A, B, C, Y


def polar_problem(n: int, seed: int = 52):
    """(X, Q, P) as complex numpy arrays with X = Q P, Q unitary, P = Z^H Z."""
    rng = np.random.default_rng(seed)
    U, R = np.linalg.qr(_uniform_complex(rng, (n, n)))
    Z = _uniform_complex(rng, (n, n))
    P = Z.conj().T @ Z
    return U @ P, U, P


def spd_pair(n: int, seed: int = 53):
    """A, B symmetric positive definite (M = A + iB complex symmetric)."""
    rng = np.random.default_rng(seed)
    G1 = rng.standard_normal((n, n))
    G2 = rng.standard_normal((n, n))
    A = G1 @ G1.T / n + np.eye(n)
    B = G2 @ G2.T / n + np.eye(n)
    return np.ascontiguousarray(0.5 * (A + A.T)), np.ascontiguousarray(0.5 * (B + B.T))
