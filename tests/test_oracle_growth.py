"""Pins of the oracle's growth ODEs (eq. d1, eq. full-d2) and the k tables.

Pins (closed forms and independent integrals, not the oracle's own formulas):
  * Einstein-de Sitter GR: D1 = a, D2(T1) = -3/7 a^2;
  * EdS with constant mu = 4/3 (a test model): D1 = a^p, p = (-1 + sqrt 33)/4,
    D2 = -2/(4p^2 + p - 2) a^{2p};
  * LCDM D1 against Heath's integral D ~ H(a) int_0^a da'/(a' H(a'))^3
    (scipy quad, an independent quadrature of a different formula);
  * LCDM D2 / (-3/7 D1^2) against the Bouchet et al. fit Omega_m^-1/143 (loose);
  * k -> 0: the f(R) solution tends to GR;
  * exact scaling: mu and the M2 term depend on k only through k^2 |f_R0|,
    so D(k; f) = D(k sqrt(f/f'); f');
  * the linear-growth enhancement of the paper's first figure is ordered
    F4 > F5 > F6 and grows with k (qualitative).
"""
import math

import numpy as np
import pytest
from scipy import integrate

import oracle
from oracle import cosmology as cz
from oracle import growth


def test_eds_gr_closed_form():
    m = oracle.Model(omega_m=1.0, gravity="gr", factorisation="t1")
    k = np.array([1e-3, 0.1, 1.0])
    for a in (1.0, 0.5, 0.1):
        d1, d2 = growth.solve(k, a, m)
        assert np.max(np.abs(d1 / a - 1)) < 1e-11
        assert np.max(np.abs(d2 / (-3 / 7 * a * a) - 1)) < 1e-10


def test_eds_constant_mu_power_law():
    mu0 = 4.0 / 3.0
    m = oracle.Model(omega_m=1.0, gravity="mu_const", mu_const=mu0, factorisation="t1")
    p = (-1 + math.sqrt(33)) / 4
    c = -2 / (4 * p * p + p - 2)
    assert abs(c + 0.415467) < 1e-6
    for a in (1.0, 0.3):
        d1, d2 = growth.solve(np.array([0.05]), a, m)
        assert abs(d1[0] / a ** p - 1) < 1e-10
        assert abs(d2[0] / (c * a ** (2 * p)) - 1) < 1e-10


def heath_growth(a, m):
    e = lambda x: math.sqrt(cz.e2(x, m))
    val, _ = integrate.quad(lambda x: 1.0 / (x * e(x)) ** 3, 0.0, a, epsabs=0, epsrel=1e-13, limit=200)
    return e(a) * val


@pytest.mark.parametrize("a", [0.5, 0.25])
def test_lcdm_d1_matches_heath_integral(a):
    m = oracle.Model(omega_m=0.3, gravity="gr", factorisation="eds")
    kn, d1, _ = growth.tables(m.with_(nk=4), a)
    ref = heath_growth(a, m) / heath_growth(1.0, m)
    assert np.max(np.abs(d1 / ref - 1)) < 1e-7


def test_lcdm_d2_near_bouchet_fit():
    m = oracle.Model(omega_m=0.3, gravity="gr", factorisation="t1", nk=4)
    _, d1, d2 = growth.tables(m, 1.0)
    ratio = d2[0] / (-3 / 7 * d1[0] ** 2)
    fit = 0.3 ** (-1 / 143)
    assert abs(ratio / fit - 1) < 1e-3
    assert ratio > 1.0


def test_fr_small_k_tends_to_gr():
    fr = oracle.Model(gravity="fr_hs", fr0_abs=1e-4, factorisation="t1")
    gr = fr.with_(gravity="gr")
    d1f, d2f = growth.solve(np.array([1e-8]), 1.0, fr)
    d1g, d2g = growth.solve(np.array([1e-8]), 1.0, gr)
    assert abs(d1f[0] / d1g[0] - 1) < 1e-12
    assert abs(d2f[0] / d2g[0] - 1) < 1e-12


def test_fr_scaling_invariance():
    f4 = oracle.Model(gravity="fr_hs", fr0_abs=1e-4, factorisation="t1")
    f6 = f4.with_(fr0_abs=1e-6)
    d1a, d2a = growth.solve(np.array([1.0]), 1.0, f6)
    d1b, d2b = growth.solve(np.array([0.1]), 1.0, f4)
    assert abs(d1a[0] / d1b[0] - 1) < 1e-11
    assert abs(d2a[0] / d2b[0] - 1) < 1e-11


def test_linear_enhancement_ordering():
    base = oracle.Model(omega_m=0.31345, h=0.6731, gravity="fr_hs", factorisation="eds", nk=64)
    gr = growth.tables(base.with_(gravity="gr"), 1.0)[1]
    ratios = {}
    for name, f in (("F4", 1e-4), ("F5", 1e-5), ("F6", 1e-6)):
        kn, d1, _ = growth.tables(base.with_(fr0_abs=f), 1.0)
        ratios[name] = d1 / gr
    assert abs(ratios["F4"][0] - 1) < 1e-4
    for r in ratios.values():
        assert np.all(np.diff(r) >= -1e-15)
    i = np.argmin(np.abs(kn - 0.1))
    assert ratios["F4"][i] > ratios["F5"][i] > ratios["F6"][i] > 1.0


def test_normalisation_and_gr_table():
    m = oracle.preset("C1")
    kn, d1, d2 = growth.tables(m, 1.0)
    assert np.all(d1 == 1.0)
    assert np.allclose(d2, -3 / 7, rtol=0, atol=1e-16)


def test_interpolation_nodes_and_clamp():
    m = oracle.Model(nk=8)
    kn = growth.nodes(m)
    assert abs(kn[0] / m.kmin - 1) < 1e-14 and abs(kn[-1] / m.kmax - 1) < 1e-14
    tab = np.linspace(0.0, 7.0, 8)
    assert np.allclose(growth.interp(kn, tab, kn, m), tab, atol=1e-12)
    mid = np.sqrt(kn[2] * kn[3])
    assert abs(growth.interp(kn, tab, mid, m) - 2.5) < 1e-12
    assert growth.interp(kn, tab, 1e-9, m) == 0.0
    assert growth.interp(kn, tab, 1e9, m) == 7.0


def test_t1_brace_reduces_in_gr():
    gr = oracle.Model(gravity="gr")
    for th in (90.0, 60.0, 80.0):
        c = growth.cos_deg(th)
        k1, k2 = growth.triangle_sides(np.array([0.3]), 1.3, c)
        b = growth.source_brace(np.array([0.3]), k1, k2, c, 0.7, gr)
        assert abs(b[0] - (1 - c * c)) < 1e-15


def test_triangle_sides_close():
    for r, th in ((1.0, 90.0), (2.0, 70.0), (1e-3, 90.0)):
        c = growth.cos_deg(th)
        k1, k2 = growth.triangle_sides(np.array([0.2]), r, c)
        assert abs(math.sqrt(k1[0] ** 2 + k2[0] ** 2 + 2 * k1[0] * k2[0] * c) - 0.2) < 1e-15
