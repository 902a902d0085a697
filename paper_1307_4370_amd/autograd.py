"""Phi as a differentiable torch operation whose backward is Phi^dagger.

For y = Phi x, the vector-Jacobian product of a real loss is Phi^dagger applied
to the output gradient (torch's conjugate-Wirtinger convention for complex
tensors); for a real input x the gradient is its real part.  Both directions run
in the HIP library.
"""
from __future__ import annotations

import torch

from ._lib import Plan


class PhiFn(torch.autograd.Function):
    """y[b] = Phi_b x[b] for a batch of images and one plan per batch item."""

    @staticmethod
    def forward(ctx, x: torch.Tensor, plans):
        plans = list(plans)
        if x.dim() != 3 or x.shape[0] != len(plans):
            raise ValueError("x must be (B, n, n) with one plan per batch item")
        ctx.plans = plans
        ctx.real_input = not x.is_complex()
        cd = plans[0].cdtype
        xc = x.to(cd)
        return torch.stack([p.phi(xc[b].contiguous()) for b, p in enumerate(plans)])

    @staticmethod
    def backward(ctx, gy: torch.Tensor):
        gy = gy.contiguous()
        gx = torch.stack([p.phi_adj(gy[b].contiguous()) for b, p in enumerate(ctx.plans)])
        if ctx.real_input:
            gx = gx.real
        return gx, None


def phi(x: torch.Tensor, plans) -> torch.Tensor:
    """Differentiable y = Phi x (batched, one plan per item)."""
    if isinstance(plans, Plan):
        plans = [plans]
    return PhiFn.apply(x, plans)
