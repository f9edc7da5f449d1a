"""Gradients of the 2LPT pipeline w.r.t. the white noise (autograd on the oracle).

Test infrastructure only (FP64 CPU oracle).  torch autograd differentiates
the oracle's own FP64 chain (its own real DFTs, pointwise multipliers, the
quadratic source and the CIC paint); no hand-written adjoint lives here, so
this is an independent check of the GPU's hand-written backward pass.
"""
from __future__ import annotations

import torch

from . import cic, fields
from .model import Model


def vjp_displace(w, g_psi1, g_psi2, m: Model, a: float, tab=None):
    """d/dw of sum(g_psi1 * psi1 + g_psi2 * psi2)."""
    w = fields.as_f64(w).clone().requires_grad_(True)
    p1, p2 = fields.displace(w, m, a, tab)
    obj = (fields.as_f64(g_psi1) * p1).sum() + (fields.as_f64(g_psi2) * p2).sum()
    obj.backward()
    return w.grad.detach()


def vjp_paint(disp, g_delta, m: Model):
    """d/d(disp) of sum(g_delta * delta_CIC(disp))."""
    d = fields.as_f64(disp).clone().requires_grad_(True)
    obj = (fields.as_f64(g_delta) * cic.paint(d, m)).sum()
    obj.backward()
    return d.grad.detach()


def loss_and_grad(w, target, m: Model, a: float, tab=None):
    """(loss, d loss / d w) for the CIC field-level loss."""
    w = fields.as_f64(w).clone().requires_grad_(True)
    p1, p2 = fields.displace(w, m, a, tab)
    val = cic.loss(cic.paint(p1 + p2, m), fields.as_f64(target))
    val.backward()
    return float(val.detach()), w.grad.detach()


def loss_value(w, target, m: Model, a: float, tab=None) -> float:
    with torch.no_grad():
        p1, p2 = fields.displace(fields.as_f64(w), m, a, tab)
        return float(cic.loss(cic.paint(p1 + p2, m), fields.as_f64(target)))
