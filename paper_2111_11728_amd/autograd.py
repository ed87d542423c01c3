"""Compliance c(rho) = f^T u(rho) of the SIMP system (Sec. 1, Eq. 1-2) as a torch autograd
function. The forward pass calls ``feti_compliance_and_grad``: it sets the context up for rho,
solves with the FETI method of the context, and writes c together with the adjoint gradient
dc/drho_e = -p rho_e^(p-1) (E0 - Emin) u_e^T K0 u_e (compliance is self-adjoint). The backward
pass scales that gradient; it does no extra solve. A solve that misses its tolerance raises
``FetiError`` in the forward pass, so no compliance or gradient of an unconverged solve reaches
autograd. Argument marshalling only: all arithmetic runs in the HIP library.
"""
from __future__ import annotations

import torch

from .feti import Context


class Compliance(torch.autograd.Function):
    @staticmethod
    def forward(ctx, rho: torch.Tensor, fctx: Context, f: torch.Tensor) -> torch.Tensor:
        if rho.dtype != torch.float64 or f.dtype != torch.float64:
            raise TypeError("rho and f must be float64")
        rho_c = rho.detach().contiguous()
        c = torch.zeros(1, dtype=torch.float64, device=rho.device)
        g = torch.empty_like(rho_c)
        fctx.feti_compliance_and_grad(rho_c, f.contiguous(), c, g)
        ctx.save_for_backward(g)
        return c[0]

    @staticmethod
    def backward(ctx, grad_c):
        (g,) = ctx.saved_tensors
        return grad_c * g, None, None


def compliance(rho: torch.Tensor, fctx: Context, f: torch.Tensor) -> torch.Tensor:
    """c(rho) with autograd support (gradient w.r.t. rho only)."""
    return Compliance.apply(rho, fctx, f)


class BatchedCompliance(torch.autograd.Function):
    """Compliances c_d(rho) of the designs of a batched context (one entry per design); rho and
    the gradient concatenate the designs. Backward scales each design's gradient block by its
    own upstream gradient."""

    @staticmethod
    def forward(ctx, rho: torch.Tensor, fctx, f: torch.Tensor) -> torch.Tensor:
        if rho.dtype != torch.float64 or f.dtype != torch.float64:
            raise TypeError("rho and f must be float64")
        rho_c = rho.detach().contiguous()
        nd = len(fctx.layout)
        c = torch.zeros(nd, dtype=torch.float64, device=rho.device)
        g = torch.empty_like(rho_c)
        fctx.feti_compliance_and_grad(rho_c, f.contiguous(), c, g)
        counts = torch.tensor([lay["n_el"] for lay in fctx.layout], device=rho.device)
        ctx.save_for_backward(g, counts)
        return c

    @staticmethod
    def backward(ctx, grad_c):
        g, counts = ctx.saved_tensors
        return torch.repeat_interleave(grad_c, counts) * g, None, None


def batched_compliance(rho: torch.Tensor, fctx, f: torch.Tensor) -> torch.Tensor:
    """[c_d(rho)] over the designs of a BatchedContext, with autograd support."""
    return BatchedCompliance.apply(rho, fctx, f)
