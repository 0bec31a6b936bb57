"""Write sampled columns of the oracle's inverse for the full-size workloads.

Calls only the FP64 CPU oracle (and the seeded input generators): the complex
Gaussian elimination of Algorithm 4 for the n = 4096 general matrix (A, B iid
N(0, 1), seed 0) and the complex Cholesky inversion of Algorithm 8 for the
n = 4096 HPD matrix (Z Z^H + n I, seed 1).  The full inverses are too large to
store, so a seeded set of columns is kept (tests compare the GPU result on
exactly these columns).  The spectral condition numbers of M, A and
C = A + B A^{-1} B are recorded as metadata for the tolerance derivation (they
are properties of the input, computed with LAPACK).

Usage: python tests/golden/make_full_size_samples.py [n] [--general-only]

--general-only writes the general matrix's columns alone, without the
condition numbers (used for n = 8192, where they would take far longer than
the inversion).
"""
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

import oracle  # noqa: E402
from paper_2208_01239_amd import inputs  # noqa: E402

HERE = os.path.dirname(os.path.abspath(__file__))


def main(n=4096, general_only=False):
    rng = np.random.default_rng(2208)
    cols = np.sort(rng.choice(n, size=8, replace=False))
    # general matrix: oracle complex LU (Algorithm 4)
    A, B = inputs.general(n, 0)
    t = time.time()
    Xr, Xi, info, _, _ = oracle.cinv_lu(A, B)
    assert info == 0
    print(f"general n={n}: oracle Algorithm 4 in {time.time() - t:.1f} s", flush=True)
    if general_only:
        np.savez_compressed(os.path.join(HERE, f"n{n}_general_samples.npz"), cols=cols, xr=Xr[:, cols],
                            xi=Xi[:, cols], a00=A[0, :4], b00=B[0, :4])
        return
    kM = float(np.linalg.cond(A + 1j * B))
    kA = float(np.linalg.cond(A))
    C = A + B @ np.linalg.solve(A, B)
    kC = float(np.linalg.cond(C))
    np.savez_compressed(os.path.join(HERE, f"n{n}_general_samples.npz"), cols=cols, xr=Xr[:, cols], xi=Xi[:, cols],
                        a00=A[0, :4], b00=B[0, :4], kappa_M=kM, kappa_A=kA, kappa_C=kC)
    del Xr, Xi, C
    # HPD matrix: oracle complex Cholesky inversion (Algorithm 8)
    A, B = inputs.hpd(n, 1)
    t = time.time()
    Xr, Xi, info, _ = oracle.cinv_chol(A, B)
    assert info == 0
    print(f"hpd n={n}: oracle Algorithm 8 in {time.time() - t:.1f} s", flush=True)
    np.savez_compressed(os.path.join(HERE, f"n{n}_hpd_samples.npz"), cols=cols, xr=Xr[:, cols], xi=Xi[:, cols],
                        a00=A[0, :4], b00=B[0, :4])
    print("kappa M %.3e A %.3e C %.3e" % (kM, kA, kC), flush=True)


if __name__ == "__main__":
    args = [a for a in sys.argv[1:] if not a.startswith("--")]
    main(int(args[0]) if args else 4096, general_only="--general-only" in sys.argv)
