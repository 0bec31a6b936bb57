"""Write oracle samples of the inverse for the large-order workloads: one
column in every 64-column band (so every panel of the blocked factorizations
owns a sampled column) and, of those columns, a fixed seeded set of 256 rows.

Calls only the FP64 CPU oracle and the seeded input generators.  Each column
x_j = M^{-1} e_j comes from complex Gaussian elimination with partial pivoting
(the factorization of Algorithm 4) followed by iterative refinement whose
residual e_j - M x_j is accumulated in double-double, so the stored values are
accurate to about the unit roundoff even where u kappa(M) is 1e-10
(kappa = 1e6).  The size of the final correction is recorded as evidence of
convergence.

The input's SHA-256 (of the raw FP64 bytes of A and B, row-major) is stored
beside the samples: the tests rebuild the matrix on the device and compare
digests before comparing values, so a matrix that is not bit-identical to the
one the oracle saw is reported as such and never graded.  The rotation-built
spectrum inputs are bit-reproducible on any device by construction; the iid
Gaussian inputs are too (numpy PCG64 draws).  The n = 4096 HPD input is
formed with a BLAS product and its digest may differ between hosts; its test
then falls back to a tolerance that covers an input perturbation of a few
units of roundoff.

Usage: python tests/golden/make_band_samples.py [case ...]   (default: all)
"""
import hashlib
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

import oracle  # noqa: E402
from paper_2208_01239_amd import inputs  # noqa: E402

HERE = os.path.dirname(os.path.abspath(__file__))
N_ROWS = 256
BAND = 64


def _cases():
    c = {
        "n4096_general": lambda: inputs.general(4096, 0),
        "n4096_hpd": lambda: inputs.hpd(4096, 1),
        "n8192_general": lambda: inputs.general(8192, 0),
    }
    for kind, base in (("general", 300), ("hpd", 400)):
        for k in (2, 4, 6):
            c[f"n8192_rot_{kind}_k1e{k}"] = (lambda kind=kind, k=k, base=base:
                                             inputs.spectrum_rotations(8192, 10.0 ** k, kind, seed=base + k))
    return c


CASES = _cases()


def digest(a: np.ndarray) -> str:
    return hashlib.sha256(np.ascontiguousarray(a, dtype=np.float64).tobytes()).hexdigest()


def sample_positions(n: int):
    rng = np.random.default_rng(2208 + n)
    cols = np.arange(0, n, BAND) + rng.integers(0, BAND, (n + BAND - 1) // BAND)
    cols = cols[cols < n]
    rows = np.sort(rng.choice(n, size=min(N_ROWS, n), replace=False))
    return cols, rows


def write_case(name: str) -> None:
    t = time.time()
    A, B = CASES[name]()
    n = A.shape[0]
    print(f"{name}: input built in {time.time() - t:.1f} s", flush=True)
    cols, rows = sample_positions(n)
    E = np.zeros((n, cols.size))
    E[cols, np.arange(cols.size)] = 1.0
    t = time.time()
    Xr, Xi, info, last = oracle.csolve_refined(A, B, E, np.zeros_like(E), steps=3)
    assert info == 0, info
    print(f"{name}: {cols.size} columns in {time.time() - t:.1f} s, final correction {last:.2e}", flush=True)
    np.savez_compressed(os.path.join(HERE, f"{name}_band_samples.npz"), cols=cols, rows=rows,
                        xr=Xr[rows], xi=Xi[rows], sha_a=digest(A), sha_b=digest(B), last_correction=last,
                        refine_steps=3)


if __name__ == "__main__":
    names = sys.argv[1:] or list(CASES)
    for nm in names:
        write_case(nm)
