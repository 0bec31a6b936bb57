"""GPU parity of the adjoint (reverse-mode derivative of the inversion),
dM = -X^H G X^H formed with Gauss's three-multiplication complex products:
against the oracle's direct complex triple loops (on seeded random X, G: the
adjoint is defined for any X), against central finite differences of
L = Re tr(W X(M)) through the GPU inversion (G = W^H), and through
torch.autograd (full Jacobian check by finite differences at n = 4)."""
import numpy as np
import pytest

import oracle
from _helpers import relF

pytestmark = pytest.mark.gpu

U32 = 2.0 ** -24


@pytest.fixture(scope="module")
def h():
    import paper_2208_01239_amd as fi
    hd = fi.Handle(0)
    yield hd
    hd.close()


def _rand(batch, n, seed):
    rng = np.random.default_rng(seed)
    return [rng.standard_normal((batch, n, n)) for _ in range(4)]


def _gpu_adjoint(h, Xr, Xi, Gr, Gi, dtype):
    import torch
    import paper_2208_01239_amd as fi
    t = [torch.from_numpy(np.ascontiguousarray(a)).to(dtype).cuda() for a in (Xr, Xi, Gr, Gi)]
    dMr, dMi = fi.frob_inv_adjoint(h, *t)
    return dMr.double().cpu().numpy(), dMi.double().cpu().numpy()


@pytest.mark.parametrize("n,batch", [(1, 3), (17, 3), (64, 2), (130, 2), (256, 2)])
def test_adjoint_fp64_matches_oracle(h, n, batch):
    import torch
    Xr, Xi, Gr, Gi = _rand(batch, n, 500 + n)
    dMr, dMi = _gpu_adjoint(h, Xr, Xi, Gr, Gi, torch.float64)
    for b in range(batch):
        Rr, Ri = oracle.adjoint(Xr[b], Xi[b], Gr[b], Gi[b])
        e = relF(dMr[b], dMi[b], Rr, Ri)
        assert e <= 1e-12, (b, e)


@pytest.mark.parametrize("n,batch", [(17, 3), (64, 2), (256, 2)])
def test_adjoint_fp32_matches_oracle(h, n, batch):
    """FP32 storage and FP32 matrix-core GEMMs: the inputs are rounded to FP32
    first (the oracle sees the same rounded values); each real product of
    length n accumulates at most n u32 relative error, and the three-product
    combinations of Gauss's scheme add a small constant factor."""
    import torch
    Xr, Xi, Gr, Gi = [a.astype(np.float32).astype(np.float64) for a in _rand(batch, n, 700 + n)]
    dMr, dMi = _gpu_adjoint(h, Xr, Xi, Gr, Gi, torch.float32)
    tol = 8 * n * U32
    for b in range(batch):
        Rr, Ri = oracle.adjoint(Xr[b], Xi[b], Gr[b], Gi[b])
        e = relF(dMr[b], dMi[b], Rr, Ri)
        print(f"n={n} b={b}: FP32 adjoint relF {e:.2e} (tol {tol:.1e})")
        assert e <= tol


@pytest.mark.parametrize("dtype_name", ["float64", "float32"])
def test_adjoint_large_batch_sampled_entries(h, dtype_name):
    """A batch large enough for the batched products' big tile: 256 entries of
    order 200 give 1024 tiles of 128 x 128, ragged in both directions, with
    the batch folded into the grid's x axis so the entries spread over every
    XCD.  Sampled entries (the first two, a middle one, the last two) against
    the oracle, at the tolerances of the tests above."""
    import torch
    dtype = getattr(torch, dtype_name)
    n, batch = 200, 256
    Xr, Xi, Gr, Gi = _rand(batch, n, 900)
    if dtype == torch.float32:
        Xr, Xi, Gr, Gi = [a.astype(np.float32).astype(np.float64) for a in (Xr, Xi, Gr, Gi)]
    dMr, dMi = _gpu_adjoint(h, Xr, Xi, Gr, Gi, dtype)
    tol = 1e-12 if dtype == torch.float64 else 8 * n * U32
    for b in (0, 1, 127, 254, 255):
        Rr, Ri = oracle.adjoint(Xr[b], Xi[b], Gr[b], Gi[b])
        e = relF(dMr[b], dMi[b], Rr, Ri)
        print(f"{dtype_name} b={b}: adjoint relF {e:.2e} (tol {tol:.1e})")
        assert e <= tol, (b, e)


def _loss(h, A, B, Wr, Wi, hpd):
    """L = Re tr(W X) with X = (A + iB)^{-1} from the GPU inversion (FP64)."""
    import torch
    import paper_2208_01239_amd as fi
    f = fi.frob_inv_hpd if hpd else fi.frob_inv_general
    Xr, Xi, _ = f(h, torch.from_numpy(A).cuda(), torch.from_numpy(B).cuda())
    Xr, Xi = Xr.cpu().numpy(), Xi.cpu().numpy()
    return float(np.sum(Wr * Xr.T) - np.sum(Wi * Xi.T)), Xr, Xi


@pytest.mark.parametrize("hpd", [False, True])
def test_adjoint_central_differences(h, hpd):
    """Re tr(dM^H E) against (L(M + hE) - L(M - hE)) / 2h, h = 1e-6, FP64, for
    eight seeded directions E (Hermitian when M is HPD)."""
    import torch
    from paper_2208_01239_amd import inputs
    n = 8
    A, B = inputs.hpd(n, 11) if hpd else inputs.general(n, 11)
    rng = np.random.default_rng(12)
    Wr, Wi = rng.standard_normal((n, n)), rng.standard_normal((n, n))
    L0, Xr, Xi = _loss(h, A, B, Wr, Wi, hpd)
    # G = W^H
    dMr, dMi = _gpu_adjoint(h, Xr[None], Xi[None], Wr.T.copy()[None], -Wi.T.copy()[None], torch.float64)
    dMr, dMi = dMr[0], dMi[0]
    step = 1e-6
    for k in range(8):
        Er, Ei = rng.standard_normal((n, n)), rng.standard_normal((n, n))
        if hpd:
            Er, Ei = 0.5 * (Er + Er.T), 0.5 * (Ei - Ei.T)
        Lp = _loss(h, A + step * Er, B + step * Ei, Wr, Wi, hpd)[0]
        Lm = _loss(h, A - step * Er, B - step * Ei, Wr, Wi, hpd)[0]
        fd = (Lp - Lm) / (2 * step)
        an = float(np.sum(dMr * Er) + np.sum(dMi * Ei))
        assert abs(fd - an) <= 1e-6 * max(1.0, abs(an)), (k, fd, an)


def test_autograd_full_jacobian(h):
    """torch.autograd.gradcheck: every entry of the Jacobian of (Mr, Mi) -> (Xr, Xi)
    by central differences against the adjoint's vector-Jacobian products."""
    import torch
    from paper_2208_01239_amd.autograd import FrobeniusInverse
    rng = np.random.default_rng(13)
    Mr = torch.from_numpy(rng.standard_normal((2, 4, 4))).cuda().requires_grad_(True)
    Mi = torch.from_numpy(rng.standard_normal((2, 4, 4))).cuda().requires_grad_(True)
    assert torch.autograd.gradcheck(lambda a, b: FrobeniusInverse.apply(a, b, h, False), (Mr, Mi),
                                    eps=1e-6, atol=1e-7, rtol=1e-6)


def test_autograd_loss_gradient(h):
    """L = sum_b Re tr(W_b X_b) on a small HPD batch: the autograd gradient equals
    the oracle's -X^H W^H X^H with X from the oracle's complex Cholesky inversion."""
    import torch
    from paper_2208_01239_amd import inputs
    from paper_2208_01239_amd.autograd import frobenius_inverse
    mats, ws = inputs.adjoint_batch(count=3, n=24, seed=5)
    A = torch.from_numpy(np.stack([m[0] for m in mats])).cuda().requires_grad_(True)
    B = torch.from_numpy(np.stack([m[1] for m in mats])).cuda().requires_grad_(True)
    Wr = torch.from_numpy(np.stack([w[0] for w in ws])).cuda()
    Wi = torch.from_numpy(np.stack([w[1] for w in ws])).cuda()
    Xr, Xi = frobenius_inverse(A, B, h, hpd=True)
    # Re tr(W X) = sum_ij (Wr_ij Xr_ji - Wi_ij Xi_ji)
    L = (Wr * Xr.transpose(1, 2)).sum() - (Wi * Xi.transpose(1, 2)).sum()
    L.backward()
    for b in range(3):
        Xor, Xoi = oracle.cinv_chol(mats[b][0], mats[b][1])[:2]
        Rr, Ri = oracle.adjoint(Xor, Xoi, ws[b][0].T.copy(), -ws[b][1].T.copy())
        e = relF(A.grad[b].cpu().numpy(), B.grad[b].cpu().numpy(), Rr, Ri)
        assert e <= 1e-10, (b, e)


def test_autograd_forward_batched_precisions(h):
    """The forward pass runs as one batched launch in the batch's precision:
    an FP32 HPD batch (Algorithm 7) matches the oracle to the FP32 bound
    16 u32 kappa_2(C), FP64 general members (Algorithm 5) to 1e-12; the
    backward pass stays in the same precision (FP32 gradient within 1e-4 of
    the oracle's: twice the forward error, about 1e-6 here, through the two
    products, plus 8 n u32 = 3e-5 for their rounding)."""
    import torch
    from paper_2208_01239_amd import inputs
    from paper_2208_01239_amd.autograd import frobenius_inverse
    mats, ws = inputs.adjoint_batch(count=4, n=64, seed=9)
    A = torch.from_numpy(np.stack([m[0] for m in mats])).float().cuda().requires_grad_(True)
    B = torch.from_numpy(np.stack([m[1] for m in mats])).float().cuda().requires_grad_(True)
    Xr, Xi = frobenius_inverse(A, B, h, hpd=True)
    assert Xr.dtype == torch.float32
    U32 = 2.0 ** -24
    for b in range(4):
        a64, b64 = (m.astype(np.float32).astype(np.float64) for m in mats[b])
        Ror, Roi = oracle.cinv_chol(a64, b64)[:2]
        kC = np.linalg.cond(a64 + b64 @ np.linalg.solve(a64, b64))
        assert relF(Xr[b].detach().cpu().numpy(), Xi[b].detach().cpu().numpy(), Ror, Roi) <= 16 * U32 * kC
    Wr = torch.from_numpy(np.stack([w[0] for w in ws])).float().cuda()
    Wi = torch.from_numpy(np.stack([w[1] for w in ws])).float().cuda()
    L = (Wr * Xr.transpose(1, 2)).sum() - (Wi * Xi.transpose(1, 2)).sum()
    L.backward()
    assert A.grad.dtype == torch.float32
    for b in range(4):
        a64, b64 = (m.astype(np.float32).astype(np.float64) for m in mats[b])
        Xor, Xoi = oracle.cinv_chol(a64, b64)[:2]
        Rr, Ri = oracle.adjoint(Xor, Xoi, ws[b][0].astype(np.float32).T.astype(np.float64).copy(),
                                -ws[b][1].astype(np.float32).T.astype(np.float64).copy())
        assert relF(A.grad[b].cpu().numpy(), B.grad[b].cpu().numpy(), Rr, Ri) <= 1e-4
    G = [inputs.general(40, 900 + b) for b in range(3)]
    Ag = torch.from_numpy(np.stack([g[0] for g in G])).cuda()
    Bg = torch.from_numpy(np.stack([g[1] for g in G])).cuda()
    Xr, Xi = frobenius_inverse(Ag, Bg, h)
    for b in range(3):
        Ror, Roi = oracle.cinv_lu(*G[b])[:2]
        assert relF(Xr[b].cpu().numpy(), Xi[b].cpu().numpy(), Ror, Roi) <= 1e-12


def test_autograd_forward_reports_failing_member(h):
    """A member with a singular real part (the batched path has no shift)
    raises, naming the member and the stage."""
    import torch
    import paper_2208_01239_amd as fi
    from paper_2208_01239_amd.autograd import frobenius_inverse
    A = torch.eye(3, dtype=torch.float64).repeat(2, 1, 1).cuda()
    B = torch.zeros_like(A)
    A[1, 0, 0] = 0.0
    B[1, 0, 0] = 1.0      # member 1 is diag(i, 1, 1): invertible, but its real part is singular
    with pytest.raises(fi.FrobSingularError, match="member 1, stage 1"):
        frobenius_inverse(A, B, h)
