"""Pins of the oracle's field pipeline (delta -> psi1, phi_,ij, S, S(k), psi2).

Closed forms used (mathematics, not the paper's numbers):
  * one plane wave delta = A cos(k.x): S = 0 and psi2 = 0, psi1 = -A D1 k sin(k.x)/k^2;
  * two plane waves A cos(ka.x) + B cos(kb.x): S = A B (1 - (ka^.kb^)^2) cos(ka.x) cos(kb.x),
    psi2 = (A B/2)(1 - c^2) sum_{+-} D2(|k+-|) k+- sin(k+-.x)/|k+-|^2;
  * <S> = 0 exactly for any field (S(k=0) collects k1 = -k2 pairs, weight 1 - c^2 = 0);
  * divergence identities i k.F[psi1] = -D1 delta, i k.F[psi2] = D2 S(k) and zero curl.
"""
import math

import numpy as np
import torch

import oracle
from oracle import fields, growth
from seeded_inputs import white_noise


def _grid(m):
    c = np.arange(m.n) * (m.box / m.n)
    return np.meshgrid(c, c, c, indexing="ij")


def _model():
    # constant-mu test model with Omega_m = 1 gives smooth, k-independent growth
    return oracle.Model(n=16, box=100.0, gravity="fr_hs", fr0_abs=1e-5, factorisation="t1")


def _dk_from_real(x, m):
    return torch.fft.rfftn(torch.from_numpy(x)) * torch.from_numpy(fields.mask(m.n))


def test_single_plane_wave_has_no_second_order():
    m = _model()
    X, Y, Z = _grid(m)
    f = 2 * math.pi / m.box
    kv = f * np.array([1.0, 2.0, -1.0])
    x = 0.7 * np.cos(kv[0] * X + kv[1] * Y + kv[2] * Z)
    tab = growth.tables(m, 1.0)
    dk = _dk_from_real(x, m)
    s = fields.source(dk, m)
    assert s.abs().max().item() < 1e-15
    p1, p2 = fields.displace_from_delta_k(dk, m, 1.0, tab)
    assert p2.abs().max().item() < 1e-14
    kk = math.sqrt(kv @ kv)
    d1 = float(growth.interp(tab[0], tab[1], kk, m))
    ph = kv[0] * X + kv[1] * Y + kv[2] * Z
    for i in range(3):
        ref = -0.7 * d1 * kv[i] * np.sin(ph) / kk ** 2
        assert np.max(np.abs(p1[i].numpy() - ref)) < 1e-12 * (0.7 * d1 / kk)


def test_two_plane_waves_closed_form():
    m = _model()
    X, Y, Z = _grid(m)
    f = 2 * math.pi / m.box
    ka = f * np.array([1.0, 0.0, 2.0])
    kb = f * np.array([0.0, -3.0, 1.0])
    A, B = 0.8, -0.5
    pa = ka[0] * X + ka[1] * Y + ka[2] * Z
    pb = kb[0] * X + kb[1] * Y + kb[2] * Z
    x = A * np.cos(pa) + B * np.cos(pb)
    dk = _dk_from_real(x, m)
    c = (ka @ kb) / math.sqrt((ka @ ka) * (kb @ kb))
    s_ref = A * B * (1 - c * c) * np.cos(pa) * np.cos(pb)
    s = fields.source(dk, m).numpy()
    assert np.max(np.abs(s - s_ref)) < 1e-13 * abs(A * B)

    tab = growth.tables(m, 1.0)
    _, p2 = fields.displace_from_delta_k(dk, m, 1.0, tab)
    ref = np.zeros((3,) + X.shape)
    for sgn in (+1, -1):
        kp = ka + sgn * kb
        kn = math.sqrt(kp @ kp)
        d2 = float(growth.interp(tab[0], tab[2], kn, m))
        ph = kp[0] * X + kp[1] * Y + kp[2] * Z
        for i in range(3):
            ref[i] += 0.5 * A * B * (1 - c * c) * d2 * kp[i] * np.sin(ph) / kn ** 2
    scale = np.max(np.abs(ref))
    assert np.max(np.abs(p2.numpy() - ref)) < 1e-12 * scale


def test_mean_source_vanishes():
    m = oracle.preset("C1").with_(n=32)
    dk = fields.delta_k(white_noise(32, 1), m)
    s = fields.source(dk, m)
    assert abs(s.mean().item()) < 1e-13 * s.abs().mean().item()


def test_divergence_and_curl_identities():
    m = oracle.Model(n=24, box=96.0, gravity="fr_hs", fr0_abs=1e-4, factorisation="t1")
    a = 0.8
    tab = growth.tables(m, a)
    w = white_noise(m.n, 2)
    dk = fields.delta_k(w, m)
    p1, p2 = fields.displace(w, m, a, tab)
    d1m, d2m = fields.growth_on_modes(m, a, tab)
    kx, ky, kz, _, _ = fields.kvectors(m)
    msk = fields.mask(m.n)
    f1 = [torch.fft.rfftn(p1[i]).numpy() * msk for i in range(3)]
    f2 = [torch.fft.rfftn(p2[i]).numpy() * msk for i in range(3)]
    div1 = 1j * (kx * f1[0] + ky * f1[1] + kz * f1[2])
    ref1 = -d1m * dk.numpy()
    assert np.max(np.abs(div1 - ref1)) < 1e-11 * np.max(np.abs(ref1))
    sk = fields.source_k(fields.source(dk, m), m).numpy()
    div2 = 1j * (kx * f2[0] + ky * f2[1] + kz * f2[2])
    ref2 = d2m * sk
    assert np.max(np.abs(div2 - ref2)) < 1e-11 * np.max(np.abs(ref2))
    for f in (f1, f2):
        cx = ky * f[2] - kz * f[1]
        cy = kz * f[0] - kx * f[2]
        cz = kx * f[1] - ky * f[0]
        big = max(np.max(np.abs(g)) for g in f)
        assert max(np.max(np.abs(cx)), np.max(np.abs(cy)), np.max(np.abs(cz))) < 1e-12 * big * 2 * math.pi


def test_shaped_field_variance_matches_power_spectrum():
    # E|delta(k)|^2 = P(k) n^3 / V n^3 ... the real-space variance of delta is
    # (1/V) sum_k P(k) over kept modes; one realisation at 64^3 is within 1%.
    m = oracle.preset("C1").with_(n=64, box=256.0)
    amp = oracle.cosmology.sigma8_amplitude(m)
    dk = fields.delta_k(white_noise(m.n, 11), m, amp)
    var = torch.fft.irfftn(dk, s=(m.n,) * 3).var(unbiased=False).item()
    _, _, _, _, kk = fields.kvectors(m)
    msk = fields.mask(m.n)
    mz = fields.modes(m.n)[2]
    wgt = np.where(mz == 0, 1.0, 2.0) * msk
    p = oracle.cosmology.power(np.where(msk > 0, kk, 1.0), m, amp)
    expect = np.sum(wgt * p) / m.volume
    assert abs(var / expect - 1) < 0.02
