"""Differentiable Frobenius inversion for PyTorch.

``FrobeniusInverse.apply(Mr, Mi, handle, hpd)`` maps a batch of complex
matrices M = Mr + i Mi (separate real tensors, shape (batch, n, n)) to
X = M^{-1} = Xr + i Xi.  The forward pass is the library's Frobenius inversion
(Algorithm 5, or Algorithm 7 when ``hpd``); the backward pass is the library's
adjoint kernel, dL/dM = -X^H G X^H with G = dL/dXr + i dL/dXi (both complex
products by Gauss's three-multiplication scheme).  float32 batches are
inverted in FP64 and rounded; the adjoint then runs in FP32.
"""
from __future__ import annotations

import torch

from . import frob_inv_adjoint, frob_inv_general, frob_inv_hpd


class FrobeniusInverse(torch.autograd.Function):
    @staticmethod
    def forward(ctx, Mr, Mi, handle, hpd=False):
        if Mr.dim() != 3 or Mr.shape != Mi.shape or Mr.shape[1] != Mr.shape[2]:
            raise ValueError("expected two (batch, n, n) tensors of the same shape")
        dt = Mr.dtype
        A64 = Mr.detach().to(torch.float64).contiguous()
        B64 = Mi.detach().to(torch.float64).contiguous()
        Xr = torch.empty_like(A64)
        Xi = torch.empty_like(A64)
        inv = frob_inv_hpd if hpd else frob_inv_general
        for b in range(A64.shape[0]):
            inv(handle, A64[b], B64[b], Xr[b], Xi[b])
        Xr, Xi = Xr.to(dt), Xi.to(dt)
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
