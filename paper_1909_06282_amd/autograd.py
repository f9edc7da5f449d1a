"""torch.autograd.Function wrappers over the hand-written adjoint.

``Displace.apply(noise, plan, a)`` returns (psi1, psi2); its backward calls
lpt2_backward (which recomputes phi_,ij from the noise).  ``PaintCIC``
wraps lpt2_paint_cic and its transpose; the same gradient reaches psi1 and
psi2 because the particle position is q + psi1 + psi2.
"""
from __future__ import annotations

import torch


class Displace(torch.autograd.Function):
    @staticmethod
    def forward(ctx, noise, plan, a):
        noise = noise.contiguous()
        psi1, psi2 = plan.displace(a, noise)
        ctx.save_for_backward(noise)
        ctx.plan, ctx.a = plan, a
        return psi1, psi2

    @staticmethod
    def backward(ctx, g1, g2):
        (noise,) = ctx.saved_tensors
        n = noise.shape[0]
        shape = (3, n, n, n)
        g1 = torch.zeros(shape, dtype=noise.dtype, device=noise.device) if g1 is None else g1.contiguous()
        g2 = torch.zeros(shape, dtype=noise.dtype, device=noise.device) if g2 is None else g2.contiguous()
        return ctx.plan.backward(ctx.a, noise, g1, g2), None, None


class PaintCIC(torch.autograd.Function):
    @staticmethod
    def forward(ctx, psi1, psi2, plan):
        psi1, psi2 = psi1.contiguous(), psi2.contiguous()
        ctx.save_for_backward(psi1, psi2)
        ctx.plan = plan
        return plan.paint_cic(psi1, psi2)

    @staticmethod
    def backward(ctx, gd):
        psi1, psi2 = ctx.saved_tensors
        g = ctx.plan.paint_cic_backward(psi1, psi2, gd.contiguous())
        return g, g, None
