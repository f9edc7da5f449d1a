"""Cloud-in-cell density of displaced particles and the field-level loss.

Test infrastructure only (FP64 CPU oracle).  Not a step the paper computes on
its own: the paper turns displacements into densities through mass
conservation (eq. deltajacobian) and measures clustering from displaced
particles; the differentiable form of this pipeline paints the displaced
particles onto a mesh.

Conventions (readings): one particle per grid node at q = i L/n, a mesh of n^3
nodes at j L/n, periodic; per axis the weight of a node at distance d is
max(0, 1 - |d|/(L/n)); rho_bar = 1 particle per cell; delta = rho - 1;
loss = sum over mesh nodes of (delta - delta_target)^2.
"""
from __future__ import annotations

import torch

from .model import Model


def paint(disp: torch.Tensor, m: Model) -> torch.Tensor:
    """delta_CIC [n][n][n] for total displacements ``disp`` [3][n][n][n] (Mpc/h).

    Differentiable in ``disp`` (the weights are linear in the in-cell offset).
    """
    n = m.n
    cell = m.box / n
    ar = torch.arange(n, dtype=torch.float64)
    grid = torch.stack(torch.meshgrid(ar, ar, ar, indexing="ij"))
    u = grid + disp / cell                         # positions in cell units
    i0 = torch.floor(u)
    f = u - i0
    i0 = i0.to(torch.int64)
    rho = torch.zeros(n * n * n, dtype=torch.float64)
    for ox in (0, 1):
        for oy in (0, 1):
            for oz in (0, 1):
                wx = f[0] if ox else 1.0 - f[0]
                wy = f[1] if oy else 1.0 - f[1]
                wz = f[2] if oz else 1.0 - f[2]
                idx = (((i0[0] + ox) % n) * n + ((i0[1] + oy) % n)) * n + ((i0[2] + oz) % n)
                rho = rho.index_add(0, idx.reshape(-1), (wx * wy * wz).reshape(-1))
    return rho.reshape(n, n, n) - 1.0


def loss(delta: torch.Tensor, target: torch.Tensor) -> torch.Tensor:
    """Sum of squared residuals between painted and target density."""
    return ((delta - target) ** 2).sum()
