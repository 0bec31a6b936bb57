"""GPU parity: libfrobinv's HIP path against the FP64 CPU oracle.

Every case runs the C ABI through the ctypes binding on the same seeded inputs
as the oracle and compares element by element (relative Frobenius error).
Tolerance: 1e-10 for the FP64 path at kappa(M) <= 1e4, the parity bar for
this method; cases built to be ill-conditioned use a bound scaled by the
conditioning, stated in the test.
"""
import json
import os

import numpy as np
import pytest

import oracle
from paper_2208_01239_amd import inputs
from _helpers import relF, res_left, res_right, to_dev, to_host

pytestmark = pytest.mark.gpu
GOLD = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden")
TOL = 1e-10


@pytest.fixture(scope="module")
def h():
    import paper_2208_01239_amd as fi
    hd = fi.Handle(0)
    yield hd
    hd.close()


def gpu_general(h, A, B, ld=None, **kw):
    import paper_2208_01239_amd as fi
    Xr, Xi, res = fi.frob_inv_general(h, to_dev(A, ld), to_dev(B, ld), **kw)
    return to_host(Xr), to_host(Xi), res


def gpu_hpd(h, A, B, ld=None, **kw):
    import paper_2208_01239_amd as fi
    Xr, Xi, res = fi.frob_inv_hpd(h, to_dev(A, ld), to_dev(B, ld), **kw)
    return to_host(Xr), to_host(Xi), res


def test_config1_n128_general(h):
    """n = 128, A, B iid N(0,1), seed 0: Frobenius on the GPU vs the oracle's
    complex Gaussian elimination (Algorithm 4) and its Algorithm 5."""
    A, B = inputs.general(128, 0)
    Rr, Ri, info, _, _ = oracle.cinv_lu(A, B)
    assert info == 0
    Xr, Xi, res = gpu_general(h, A, B)
    e = relF(Xr, Xi, Rr, Ri)
    print(f"config1 relF(gpu frobenius, oracle complex LU) = {e:.3e}  res={res}")
    assert e <= TOL
    Fr, Fi, info, _ = oracle.frob_lu(A, B)
    assert relF(Xr, Xi, Fr, Fi) <= TOL
    rl, rr = res_left(A, B, Xr, Xi), res_right(A, B, Xr, Xi)
    print(f"config1 res_L={rl:.2e} res_R={rr:.2e}")
    assert rl < 1e-11 and rr < 1e-11


@pytest.mark.parametrize("n", [1, 2, 3, 7, 16, 17, 31, 63, 64, 65, 100, 127, 128, 129, 200, 255, 257, 300, 511, 513])
def test_general_sizes(h, n):
    A, B = inputs.general(n, 1000 + n)
    Rr, Ri, info, _, _ = oracle.cinv_lu(A, B)
    assert info == 0
    Xr, Xi, res = gpu_general(h, A, B)
    e = relF(Xr, Xi, Rr, Ri)
    kappa = np.linalg.cond(A + 1j * B)
    print(f"n={n} kappa={kappa:.2e} relF={e:.3e}")
    assert kappa <= 1e4
    assert e <= TOL
    assert res["mu_used"] == 0.0 and res["info"] == 0


@pytest.mark.parametrize("n,ld", [(33, 40), (130, 133), (257, 300)])
def test_general_leading_dimension(h, n, ld):
    A, B = inputs.general(n, 77 + n)
    Rr, Ri, _, _, _ = oracle.cinv_lu(A, B)
    import paper_2208_01239_amd as fi
    import torch
    Xr = torch.zeros((n, ld + 3), dtype=torch.float64, device="cuda")[:, :n]
    Xi = torch.zeros((n, ld + 3), dtype=torch.float64, device="cuda")[:, :n]
    fi.frob_inv_general(h, to_dev(A, ld), to_dev(B, ld), Xr, Xi)
    assert relF(to_host(Xr), to_host(Xi), Rr, Ri) <= TOL


@pytest.mark.parametrize("n", [1, 2, 5, 16, 63, 64, 65, 128, 129, 200, 257, 513])
def test_hpd_sizes(h, n):
    A, B = inputs.hpd(n, 2000 + n)
    Rr, Ri, info, _ = oracle.frob_chol(A, B)
    assert info == 0
    Cr, Ci, info, _, _ = oracle.cinv_lu(A, B)
    Xr, Xi, res = gpu_hpd(h, A, B)
    e = relF(Xr, Xi, Rr, Ri)
    print(f"hpd n={n} relF(gpu, oracle alg7)={e:.3e} relF(gpu, oracle alg4)={relF(Xr, Xi, Cr, Ci):.3e}")
    assert e <= TOL and relF(Xr, Xi, Cr, Ci) <= TOL
    # Lemma 4.5 applied to X^{-1}: Re X symmetric, Im X skew
    assert np.abs(Xr - Xr.T).max() <= 1e-14 * np.abs(Xr).max()
    assert np.abs(Xi + Xi.T).max() <= 1e-12 * np.abs(Xr).max()


def test_hpd_paper_accuracy_generator(h):
    """Section 5.6 accuracy generator: Q Lambda Q^H / ||Lambda||_F, kappa = 10."""
    rng = np.random.default_rng(56)
    n = 96
    Y = rng.uniform(-1, 1, (n, n)) + 1j * rng.uniform(-1, 1, (n, n))
    Q, _ = np.linalg.qr(Y)
    lam = np.concatenate([[10.0], rng.uniform(1, 10, n - 2), [1.0]])
    M = (Q * lam) @ Q.conj().T / np.linalg.norm(lam)
    M = 0.5 * (M + M.conj().T)
    A, B = M.real.copy(), M.imag.copy()
    Rr, Ri, _, _ = oracle.frob_chol(A, B)
    Xr, Xi, _ = gpu_hpd(h, A, B)
    assert relF(Xr, Xi, Rr, Ri) <= TOL
    assert res_left(A, B, Xr, Xi) < 1e-14 and res_right(A, B, Xr, Xi) < 1e-14


def test_hpd_rejects_indefinite(h):
    import paper_2208_01239_amd as fi
    A = np.diag([1.0, -1.0, 2.0])
    B = np.zeros((3, 3))
    with pytest.raises(fi.FrobNotHPDError):
        gpu_hpd(h, A, B)


def test_shift_worked_example(h):
    """diag(1, i): A and B singular; the shift recovers diag(1, -i)."""
    import paper_2208_01239_amd as fi
    g = json.load(open(os.path.join(GOLD, "diag_1_i.json")))
    A, B = np.array(g["Mr"]), np.array(g["Mi"])
    Xr, Xi, res = gpu_general(h, A, B)
    assert res["shifts_tried"] >= 1 and 0.0 < res["mu_used"] < 1.0
    assert np.abs(Xr - np.array(g["Xr"])).max() < 1e-15
    assert np.abs(Xi - np.array(g["Xi"])).max() < 1e-15
    with pytest.raises(fi.FrobSingularError) as ei:
        gpu_general(h, A, B, shift=fi.FROB_SHIFT_OFF)
    assert ei.value.result.stage == 1


@pytest.mark.parametrize("mu", [0.1, 0.5, 0.9])
def test_shift_on_matches_oracle_alg6(h, mu):
    import paper_2208_01239_amd as fi
    A, B = inputs.general(150, 66)
    Rr, Ri, info, _ = oracle.frob_shift(A, B, mu)
    assert info == 0
    Xr, Xi, res = gpu_general(h, A, B, shift=fi.FROB_SHIFT_ON, mu=mu)
    assert res["mu_used"] == mu
    assert relF(Xr, Xi, Rr, Ri) <= TOL


def test_shift_singular_real_part(h):
    rng = np.random.default_rng(5)
    n = 96
    A = rng.standard_normal((n, n))
    A[:, 3] = 0.0
    B = rng.standard_normal((n, n))
    ref = np.linalg.inv(A + 1j * B)
    Xr, Xi, res = gpu_general(h, A, B)
    assert res["shifts_tried"] >= 1
    Or, Oi, info, _ = oracle.frob_shift(A, B, res["mu_used"])
    assert info == 0
    assert relF(Xr, Xi, Or, Oi) <= TOL
    assert relF(Xr, Xi, ref.real, ref.imag) <= 1e-9


def test_singular_moore_penrose_example(h):
    import paper_2208_01239_amd as fi
    g = json.load(open(os.path.join(GOLD, "moore_penrose_3x3.json")))
    A, B = np.array(g["Mr"]), np.array(g["Mi"])
    for shift in (fi.FROB_SHIFT_OFF, fi.FROB_SHIFT_AUTO, fi.FROB_SHIFT_ON):
        with pytest.raises(fi.FrobSingularError):
            gpu_general(h, A, B, shift=shift)


@pytest.mark.parametrize("n,p", [(1, 1), (70, 1), (129, 3), (300, 70), (1100, 5)])
def test_solve(h, n, p):
    import paper_2208_01239_amd as fi
    A, B = inputs.general(n, 3000 + n)
    rng = np.random.default_rng(n)
    x0 = rng.uniform(-1, 1, (n, p))
    y0 = rng.uniform(-1, 1, (n, p))
    c = A @ x0 - B @ y0
    d = B @ x0 + A @ y0
    ox, oy, info, _ = oracle.frob_solve(A, B, c, d)
    assert info == 0
    x, y, res = fi.frob_solve(h, to_dev(A), to_dev(B), to_dev(c), to_dev(d))
    x, y = to_host(x), to_host(y)
    # The forward error of the Frobenius route is governed by kappa(C),
    # C = A + B A^{-1} B (eq. (cond1) and the discussion after Algorithm 3), not
    # by kappa(M); two correct FP64 executions differ by about u kappa(C).
    C = A + B @ np.linalg.solve(A, B)
    tol = max(TOL, 16 * np.finfo(float).eps / 2 * np.linalg.cond(C))
    e = relF(x, y, ox, oy)
    print(f"solve n={n} p={p} relF(gpu, oracle alg3)={e:.2e} tol={tol:.2e}")
    assert e <= tol
    assert relF(x, y, x0, y0) <= max(tol, 1e-9)


def test_refinement_reduces_error(h):
    """Newton-Schulz steps: the residual I - M X squares per step."""
    A, B = inputs.general(256, 91)
    Rr, Ri, _, _, _ = oracle.cinv_lu(A, B)
    X0r, X0i, _ = gpu_general(h, A, B)
    X1r, X1i, res = gpu_general(h, A, B, refine=1, refine_tol=1e-300)
    assert res["refine_steps"] == 1
    M = A + 1j * B
    r0 = np.linalg.norm(np.eye(256) - M @ (X0r + 1j * X0i))
    r1 = np.linalg.norm(np.eye(256) - M @ (X1r + 1j * X1i))
    print(f"refine: ||I-MX|| {r0:.3e} -> {r1:.3e}")
    assert r1 <= max(10 * r0 * r0, 1e-13 * 256)
    assert relF(X1r, X1i, Rr, Ri) <= TOL


def test_refinement_without_closing_residual(h):
    """Skipping the residual of the last iterate changes no arithmetic of the
    refinement: the same inverse, bit for bit, with resid reported as NaN."""
    A, B = inputs.general(256, 91)
    X1r, X1i, res1 = gpu_general(h, A, B, refine=1, refine_tol=1e-300)
    X2r, X2i, res2 = gpu_general(h, A, B, refine=1, refine_tol=1e-300, final_resid=False)
    # the norm is summed with atomics in no fixed order: equal up to rounding
    assert res2["refine_steps"] == 1 and np.isnan(res2["resid"])
    assert abs(res2["resid0"] - res1["resid0"]) <= 1e-12 * res1["resid0"]
    assert np.array_equal(X1r, X2r) and np.array_equal(X1i, X2i)


def test_determinism(h):
    A, B = inputs.general(200, 4)
    X1 = gpu_general(h, A, B)
    X2 = gpu_general(h, A, B)
    assert np.array_equal(X1[0], X2[0]) and np.array_equal(X1[1], X2[1])


# ----------------------------------------------------------------------------- complex-arithmetic baselines
def gpu_cinv(h, fn, A, B, form, ld=None):
    Xr, Xi, res = fn(h, to_dev(A, ld), to_dev(B, ld), form=form)
    return to_host(Xr), to_host(Xi), res


@pytest.mark.parametrize("form", [0, 1])
@pytest.mark.parametrize("n", [1, 2, 7, 31, 32, 33, 64, 65, 100, 129, 257, 300, 513])
def test_cinv_lu_baseline(h, n, form):
    """Algorithm 4 in complex arithmetic on the GPU vs the oracle's Algorithm 4."""
    import paper_2208_01239_amd as fi
    A, B = inputs.general(n, 4000 + n)
    Rr, Ri, info, _, _ = oracle.cinv_lu(A, B)
    assert info == 0
    Xr, Xi, _ = gpu_cinv(h, fi.frob_cinv_lu, A, B, form)
    e = relF(Xr, Xi, Rr, Ri)
    print(f"cinv_lu n={n} form={form} relF={e:.2e}")
    assert e <= TOL


@pytest.mark.parametrize("form", [0, 1])
@pytest.mark.parametrize("n", [1, 2, 5, 31, 32, 33, 64, 65, 128, 129, 257, 513])
def test_cinv_chol_baseline(h, n, form):
    """Algorithm 8 in complex arithmetic on the GPU vs the oracle's Algorithm 8."""
    import paper_2208_01239_amd as fi
    A, B = inputs.hpd(n, 5000 + n)
    Rr, Ri, info, _ = oracle.cinv_chol(A, B)
    assert info == 0
    Xr, Xi, _ = gpu_cinv(h, fi.frob_cinv_chol, A, B, form)
    e = relF(Xr, Xi, Rr, Ri)
    print(f"cinv_chol n={n} form={form} relF={e:.2e}")
    assert e <= TOL
    assert np.abs(Xr - Xr.T).max() <= 1e-13 * np.abs(Xr).max()
    assert np.abs(Xi + Xi.T).max() <= 1e-13 * np.abs(Xr).max()


def test_baselines_reject_singular_and_indefinite(h):
    import paper_2208_01239_amd as fi
    g = json.load(open(os.path.join(GOLD, "moore_penrose_3x3.json")))
    A, B = np.array(g["Mr"]), np.array(g["Mi"])
    for form in (0, 1):
        with pytest.raises(fi.FrobSingularError):
            gpu_cinv(h, fi.frob_cinv_lu, A, B, form)
        with pytest.raises(fi.FrobNotHPDError):
            gpu_cinv(h, fi.frob_cinv_chol, np.diag([1.0, -1.0, 2.0]), np.zeros((3, 3)), form)


def test_config1_frobenius_vs_gpu_complex_lu(h):
    """n = 128, seed 0: the GPU Frobenius result and the GPU complex-LU result
    both match the oracle's complex LU (configuration of the headline metric)."""
    import paper_2208_01239_amd as fi
    A, B = inputs.general(128, 0)
    Rr, Ri, _, _, _ = oracle.cinv_lu(A, B)
    Fr, Fi, _ = gpu_general(h, A, B)
    for form in (0, 1):
        Cr, Ci, _ = gpu_cinv(h, fi.frob_cinv_lu, A, B, form)
        assert relF(Cr, Ci, Rr, Ri) <= TOL
    assert relF(Fr, Fi, Rr, Ri) <= TOL


# ----------------------------------------------------------------------------- full size (n = 4096)
def _golden(name):
    path = os.path.join(GOLD, name)
    if not os.path.exists(path):
        pytest.skip(f"{name} not generated (tests/golden/make_full_size_samples.py)")
    return np.load(path, allow_pickle=False)


def test_full_size_general_n4096(h):
    """n = 4096, A, B iid N(0,1), seed 0, in the launch configuration bench.py
    times.  Sampled columns against the oracle's Algorithm 4 (stored).
    kappa(M) = 8.7e3 <= 1e4 but kappa(C) = 1.3e7: the plain FP64 Frobenius
    result is held to the kappa(C)-derived bound 16 u kappa_2(C); one
    Newton-Schulz step brings it to the 1e-10 bar."""
    g = _golden("n4096_general_samples.npz")
    n = 4096
    A, B = inputs.general(n, 0)
    assert np.array_equal(A[0, :4], g["a00"]) and np.array_equal(B[0, :4], g["b00"])
    import paper_2208_01239_amd as fi
    import torch
    cols = g["cols"]
    dA, dB = to_dev(A), to_dev(B)
    Xr, Xi, _ = fi.frob_inv_general(h, dA, dB)
    xr, xi = Xr[:, cols].cpu().numpy(), Xi[:, cols].cpu().numpy()
    e0 = relF(xr, xi, g["xr"], g["xi"])
    tol0 = 16 * np.finfo(float).eps / 2 * float(g["kappa_C"])
    Xr, Xi, res = fi.frob_inv_general(h, dA, dB, Xr, Xi, refine=1)
    xr, xi = Xr[:, cols].cpu().numpy(), Xi[:, cols].cpu().numpy()
    e1 = relF(xr, xi, g["xr"], g["xi"])
    print(f"n=4096 general: relF plain={e0:.2e} (tol {tol0:.1e}), refined={e1:.2e}; kappa M {float(g['kappa_M']):.2e} "
          f"C {float(g['kappa_C']):.2e}")
    assert e0 <= tol0
    assert e1 <= TOL
    del dA, dB, Xr, Xi
    torch.cuda.empty_cache()


def test_full_size_general_n8192(h):
    """n = 8192, the same recipe (A, B iid N(0,1), seed 0): sampled columns
    against the oracle's Algorithm 4 (stored; generated without condition
    numbers).  One Newton-Schulz step (FP32 and FP64 correction) and the
    complex-LU baseline (both forms) are held to the 1e-10 bar; the plain
    FP64 result only to 1e-7 (its error, about u kappa(C), was not bounded
    from kappa(C) here)."""
    g = _golden("n8192_general_samples.npz")
    n = 8192
    A, B = inputs.general(n, 0)
    assert np.array_equal(A[0, :4], g["a00"]) and np.array_equal(B[0, :4], g["b00"])
    import paper_2208_01239_amd as fi
    import torch
    cols = g["cols"]
    dA, dB = to_dev(A), to_dev(B)
    Xr = torch.empty_like(dA)
    Xi = torch.empty_like(dA)

    def err():
        return relF(Xr[:, cols].cpu().numpy(), Xi[:, cols].cpu().numpy(), g["xr"], g["xi"])
    fi.frob_inv_general(h, dA, dB, Xr, Xi)
    e0 = err()
    fi.frob_inv_general(h, dA, dB, Xr, Xi, refine=1, f32_correction=True)
    e32 = err()
    fi.frob_inv_general(h, dA, dB, Xr, Xi, refine=1)
    e64 = err()
    ez = []
    for form in (1, 0):
        fi.frob_cinv_lu(h, dA, dB, Xr, Xi, form=form)
        ez.append(err())
    print(f"n=8192 general: relF plain={e0:.2e}, one step FP32 / FP64 correction {e32:.2e} / {e64:.2e}; "
          f"complex LU forms 1 / 0 {ez[0]:.2e} / {ez[1]:.2e}")
    assert e0 <= 1e-7
    assert e32 <= TOL and e64 <= TOL
    assert max(ez) <= TOL
    del dA, dB, Xr, Xi
    torch.cuda.empty_cache()


def test_full_size_hpd_n4096(h):
    """n = 4096 HPD (Z Z^H + n I, seed 1): Algorithm 7 on the GPU against the
    oracle's Algorithm 8 on sampled columns, at 1e-10."""
    g = _golden("n4096_hpd_samples.npz")
    n = 4096
    A, B = inputs.hpd(n, 1)
    import paper_2208_01239_amd as fi
    import torch
    cols = g["cols"]
    Xr, Xi, _ = fi.frob_inv_hpd(h, to_dev(A), to_dev(B))
    xr, xi = Xr[:, cols].cpu().numpy(), Xi[:, cols].cpu().numpy()
    e = relF(xr, xi, g["xr"], g["xi"])
    print(f"n=4096 hpd: relF={e:.2e}")
    assert e <= TOL
    for form in (0, 1):
        Cr, Ci, _ = fi.frob_cinv_chol(h, to_dev(A), to_dev(B), form=form)
        assert relF(Cr[:, cols].cpu().numpy(), Ci[:, cols].cpu().numpy(), g["xr"], g["xi"]) <= TOL
    del Xr, Xi, Cr, Ci
    torch.cuda.empty_cache()


def test_full_size_complex_lu_n4096(h):
    g = _golden("n4096_general_samples.npz")
    A, B = inputs.general(4096, 0)
    import paper_2208_01239_amd as fi
    cols = g["cols"]
    for form in (0, 1):
        Xr, Xi, _ = fi.frob_cinv_lu(h, to_dev(A), to_dev(B), form=form)
        e = relF(Xr[:, cols].cpu().numpy(), Xi[:, cols].cpu().numpy(), g["xr"], g["xi"])
        print(f"n=4096 complex LU form {form}: relF={e:.2e}")
        assert e <= TOL


@pytest.mark.parametrize("n", [1024, 1300])
def test_lookahead_lu_orders(h, n):
    """Orders at which the LU runs in panels with a look-ahead on a second
    stream (a whole number of panels and a ragged last panel): Frobenius
    inversion and the complex-LU baseline against the oracle's inverse."""
    A, B = inputs.general(n, 77)
    Rr, Ri, info, _, _ = oracle.cinv_lu(A, B)
    assert info == 0
    C = A + B @ np.linalg.solve(A, B)
    tol = max(TOL, 16 * np.finfo(float).eps / 2 * np.linalg.cond(C))
    Xr, Xi, _ = gpu_general(h, A, B)
    e = relF(Xr, Xi, Rr, Ri)
    print(f"n={n} frobenius relF={e:.2e} tol={tol:.1e}")
    assert e <= tol
    for form in (1, 0):
        Zr, Zi, _ = gpu_cinv(h, __import__("paper_2208_01239_amd").frob_cinv_lu, A, B, form)
        ez = relF(Zr, Zi, Rr, Ri)
        print(f"n={n} complex LU form {form} relF={ez:.2e}")
        assert ez <= max(TOL, 16 * np.finfo(float).eps / 2 * np.linalg.cond(A + 1j * B))


def _backward_error_cols(A, B, xr, xi, cols):
    """||M x_j - e_j|| / (||M||_F ||x_j||) over sampled columns, in numpy FP64."""
    n = A.shape[0]
    E = np.zeros((n, len(cols)))
    E[cols, np.arange(len(cols))] = 1.0
    Rr = A @ xr - B @ xi - E
    Ri = A @ xi + B @ xr
    normM = np.sqrt(np.sum(A * A) + np.sum(B * B))
    return float(np.sqrt(np.sum(Rr ** 2 + Ri ** 2)) / (normM * np.sqrt(np.sum(xr ** 2 + xi ** 2))))


def test_large_order_n8192(h):
    """n = 8192 (the tallest leaves with a fused bottom node, 16 rows per
    thread; complex leaves of one column): M = U diag(sigma) V^H with kappa =
    1e2, drawn on the device.  Checked by properties that hold at any size:
    the backward error on sampled columns (numpy FP64 on the host), and the
    forward error against V diag(1/sigma) U^H built from the same factors
    (exact up to about kappa u)."""
    import paper_2208_01239_amd as fi
    import torch
    n = 8192
    cols = np.sort(np.random.default_rng(8192).choice(n, size=8, replace=False))

    def check(kind, fn, **kw):
        dA, dB, Rr, Ri = inputs.spectrum_device(n, 1e2, kind=kind, seed=302 + 2)
        A, B = dA.cpu().numpy(), dB.cpu().numpy()
        out = fn(h, dA, dB, **kw)
        xr, xi = out[0][:, cols].cpu().numpy(), out[1][:, cols].cpu().numpy()
        fwd = relF(xr, xi, Rr[:, cols].cpu().numpy(), Ri[:, cols].cpu().numpy())
        bwd = _backward_error_cols(A, B, xr, xi, cols)
        del dA, dB, Rr, Ri, out
        torch.cuda.empty_cache()
        return fwd, bwd

    # plain FP64 Frobenius inversion: error of forming and inverting C (about
    # u kappa(C)); its backward error is held to the same 1e-11 as Algorithm 4
    f, b = check("general", fi.frob_inv_general)
    print(f"n=8192 general plain: fwd {f:.2e} bwd {b:.2e}")
    assert b <= 1e-11 and f <= 1e-7
    f, b = check("general", fi.frob_inv_general, refine=2)
    print(f"n=8192 general refine=2: fwd {f:.2e} bwd {b:.2e}")
    assert b <= 1e-13 and f <= 1e-11
    f, b = check("hpd", fi.frob_inv_hpd)
    print(f"n=8192 hpd: fwd {f:.2e} bwd {b:.2e}")
    assert b <= 1e-13 and f <= 1e-11
    # Complex GEPP inversion (Algorithm 4) has a backward error that grows with
    # n on these matrices: the oracle's own Algorithm 4 measures 5e-15, 1.7e-14
    # and 5.6e-14 at n = 512, 1024, 2048 (about 3x per doubling), i.e. about
    # 6e-13 extrapolated to 8192; the bounds leave a factor 10 beyond that.
    f, b = check("general", fi.frob_cinv_lu, form=1)
    print(f"n=8192 complex LU: fwd {f:.2e} bwd {b:.2e}")
    assert b <= 1e-11 and f <= 1e-9
