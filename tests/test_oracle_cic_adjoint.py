"""Pins of the oracle's CIC paint, loss and autograd gradient.

  * zero displacement gives delta = 0; the total mass is conserved for any
    displacement; a particle half a cell along x splits 1/2, 1/2;
  * the autograd gradient of the loss w.r.t. the white noise agrees with
    central finite differences in FP64;
  * dot-product (adjoint) identity for the linear part: for psi1 (linear in
    w), <J v, u> = <v, J^T u> using autograd's VJP.
"""
import numpy as np
import torch

import oracle
from oracle import adjoint, cic, fields, growth
from seeded_inputs import white_noise, cell_sample


def test_cic_zero_displacement_and_mass():
    m = oracle.Model(n=8, box=16.0)
    z = torch.zeros((3, 8, 8, 8), dtype=torch.float64)
    assert cic.paint(z, m).abs().max().item() == 0.0
    rng = np.random.default_rng(0)
    d = torch.from_numpy(rng.normal(scale=5.0, size=(3, 8, 8, 8)))
    rho = cic.paint(d, m) + 1.0
    assert abs(rho.sum().item() - 512.0) < 1e-10


def test_cic_single_particle_split():
    m = oracle.Model(n=8, box=16.0)
    d = torch.zeros((3, 8, 8, 8), dtype=torch.float64)
    d[0] = 1.0                     # half a cell (cell = 2 Mpc/h) for every particle
    rho = cic.paint(d, m) + 1.0
    assert torch.allclose(rho, torch.ones_like(rho))
    d = torch.zeros((3, 8, 8, 8), dtype=torch.float64)
    d[0, 0, 0, 0] = 1.0            # one particle moved half a cell
    rho = cic.paint(d, m) + 1.0
    assert abs(rho[0, 0, 0].item() - 0.5) < 1e-15
    assert abs(rho[1, 0, 0].item() - 1.5) < 1e-15


def test_loss_gradient_matches_finite_differences():
    m = oracle.Model(n=16, box=64.0, gravity="fr_hs", fr0_abs=1e-5, factorisation="t1", nk=64)
    a = 1.0
    tab = growth.tables(m, a)
    w = white_noise(16, 5)
    with torch.no_grad():
        p1, p2 = fields.displace(white_noise(16, 7), m, a, tab)
        target = cic.paint(p1 + p2, m)
    _, g = adjoint.loss_and_grad(w, target, m, a, tab)
    eps = 1e-3
    for c in cell_sample(16, 6, seed=0):
        wp = w.copy(); wp.flat[c] += eps
        wm = w.copy(); wm.flat[c] -= eps
        fd = (adjoint.loss_value(wp, target, m, a, tab) - adjoint.loss_value(wm, target, m, a, tab)) / (2 * eps)
        gc = g.reshape(-1)[c].item()
        assert abs(fd - gc) <= 2e-4 * max(1.0, abs(gc)), (c, fd, gc)


def test_psi1_adjoint_dot_product():
    m = oracle.Model(n=12, box=48.0, gravity="fr_hs", fr0_abs=1e-5, factorisation="t1", nk=32)
    a = 1.0
    tab = growth.tables(m, a)
    rng = np.random.default_rng(1)
    v = torch.from_numpy(rng.standard_normal((12, 12, 12)))
    u = torch.from_numpy(rng.standard_normal((3, 12, 12, 12)))
    p1, _ = fields.displace(v, m, a, tab)
    lhs = (p1 * u).sum().item()
    gt = adjoint.vjp_displace(np.zeros((12, 12, 12)), u, torch.zeros_like(u), m, a, tab)
    rhs = (v * gt).sum().item()
    assert abs(lhs - rhs) < 1e-12 * abs(lhs)
