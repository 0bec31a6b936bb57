"""Differentiable Frobenius inversion for PyTorch.

``FrobeniusInverse.apply(Mr, Mi, handle, hpd)`` maps a batch of complex
matrices M = Mr + i Mi (separate real tensors, shape (batch, n, n)) to
X = M^{-1} = Xr + i Xi.  The forward pass is the library's Frobenius inversion
(Algorithm 5, or Algorithm 7 when ``hpd``): for orders up to 512 the whole
batch in one persistent batched launch in the batch's own precision (FP32 or
FP64), above that one call per matrix; the backward pass is the library's
adjoint kernel, dL/dM = -X^H G X^H with G = dL/dXr + i dL/dXi (both complex
products by Gauss's three-multiplication scheme), in the same precision.  A
member whose factorization fails raises (the batched path has no shift).
"""
from __future__ import annotations

import torch

from . import BatchedPlan, frob_inv_adjoint, frob_inv_general, frob_inv_hpd
from ._lib import FROB_NOT_HPD, FROB_SINGULAR, check


class FrobeniusInverse(torch.autograd.Function):
    @staticmethod
    def forward(ctx, Mr, Mi, handle, hpd=False):
        if Mr.dim() != 3 or Mr.shape != Mi.shape or Mr.shape[1] != Mr.shape[2]:
            raise ValueError("expected two (batch, n, n) tensors of the same shape")
        if Mr.dtype not in (torch.float32, torch.float64) or Mi.dtype != Mr.dtype:
            raise TypeError("expected float32 or float64 tensors of one dtype")
        A = Mr.detach().contiguous()
        B = Mi.detach().contiguous()
        Xr = torch.empty_like(A)
        Xi = torch.empty_like(A)
        batch, n = A.shape[0], A.shape[1]
        if batch and n <= 512:
            plan = BatchedPlan([A[b] for b in range(batch)], [B[b] for b in range(batch)], [int(hpd)] * batch,
                               [Xr[b] for b in range(batch)], [Xi[b] for b in range(batch)])
            plan.launch(handle)
            info = plan.info_dev.cpu()
            bad = torch.nonzero(info).flatten()
            if bad.numel():
                b = int(bad[0])
                w = int(info[b])
                st = FROB_NOT_HPD if hpd and w > 0 else FROB_SINGULAR
                check(st, f"FrobeniusInverse.forward (member {b}, stage {w // 1000000}, column {w % 1000000})")
        else:
            inv = frob_inv_hpd if hpd else frob_inv_general
            for b in range(batch):
                inv(handle, A[b], B[b], Xr[b], Xi[b])
        ctx.save_for_backward(Xr, Xi)
        ctx.handle = handle
        return Xr, Xi

    @staticmethod
    def backward(ctx, gXr, gXi):
        Xr, Xi = ctx.saved_tensors
        gXr = torch.zeros_like(Xr) if gXr is None else gXr.contiguous()
        gXi = torch.zeros_like(Xi) if gXi is None else gXi.contiguous()
        dMr, dMi = frob_inv_adjoint(ctx.handle, Xr, Xi, gXr.to(Xr.dtype), gXi.to(Xr.dtype))
        return dMr, dMi, None, None


def frobenius_inverse(Mr, Mi, handle, hpd=False):
    """X = (Mr + i Mi)^{-1} for a batch, differentiable with respect to Mr and Mi."""
    return FrobeniusInverse.apply(Mr, Mi, handle, hpd)
