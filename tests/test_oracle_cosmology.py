"""Pins of the oracle's background and gravity coefficients against their
definitions, evaluated here by independent routes (not the oracle's formulas
retyped):

  * the top-hat window is the Fourier transform of a uniform unit-volume
    sphere: a radial quadrature of (1/V) int_sphere exp(i k.x) d^3x;
  * sigma8: the variance of the field smoothed on 8 Mpc/h,
    int d^3k/(2 pi)^3 P(k) W^2(8k), by adaptive quadrature over k (the oracle
    uses Simpson's rule in ln k), must give the requested sigma8;
  * M1 and M2 of eq. mihusawicki are the first two derivatives of R(f_R)
    at the background (eq. mg-pot-exp).  Here R(f_R) is the exact inverse of
    f_R = df/dR for eq. husawicki (n = 1, beta^2 = H0^2 Omega_m,
    c1/c2 = 6 Omega_L/Omega_m, c2 fixed by f_R(R0) = -|f_R0|), the
    background curvature is R = 6 (dH/dt + 2 H^2) with dH/dt by finite
    differences of H(a), and the derivatives are five-point finite
    differences.  The printed coefficients take the limit c2 R/beta^2 >> 1;
    the tolerance is a few times the size of the neglected term,
    1/(c2 R/beta^2);
  * 4 pi G rho_bar(a): Friedmann's equation gives 4 pi G rho_m = (3/2) H^2
    Omega_m(a); and with the published values of G and of the critical
    density, 4 pi G rho_crit Omega_m a^-3 / c^2 in (h/Mpc)^2.

  * the BBKS transfer function: its power series at small q and in 1/q at
    large q, computed with exact rational series arithmetic (see below), and
    its dependence on k through k/(Omega_m h).
"""
import math

import numpy as np
import pytest
from scipy import integrate

import oracle
from oracle import cosmology as cz

C_KMS = 299792.458


def _h_of_a(a, m):
    """H(a) in h/Mpc from the Friedmann equation of a flat matter + Lambda
    universe (independent of the oracle's e2())."""
    h0 = 100.0 / C_KMS
    return h0 * math.sqrt(m.omega_m / a ** 3 + (1.0 - m.omega_m))


def _ricci(a, m):
    """R = 6 (dH/dt + 2 H^2) with dH/dt = a H dH/da (c = 1); dH/da by a
    five-point finite difference of H(a)."""
    eps = 1e-3 * a
    v = [_h_of_a(a + j * eps, m) for j in (-2, -1, 1, 2)]
    dh = (v[0] - 8 * v[1] + 8 * v[2] - v[3]) / (12 * eps)
    hh = _h_of_a(a, m)
    return 6.0 * (a * hh * dh + 2.0 * hh * hh)


@pytest.mark.parametrize("x", [1e-3, 0.1, 1.0, 2.5, 7.0, 20.0, 63.0])
def test_tophat_window_is_the_transform_of_a_sphere(x):
    # (1/V) int_0^R 4 pi r^2 sin(k r)/(k r) dr with R = 1, k = x
    vol = 4.0 * math.pi / 3.0
    val, _ = integrate.quad(lambda r: 4.0 * math.pi * r * math.sin(x * r) / x, 0.0, 1.0,
                            epsabs=1e-14, epsrel=1e-12, limit=400)
    assert abs(float(cz.tophat_window(x)) - val / vol) < 1e-10


@pytest.mark.parametrize("omega_m,h,n_s,sigma8", [(0.3, 0.7, 0.96, 0.8), (0.31345, 0.6731, 0.9658, 0.847)])
def test_sigma8_normalisation_by_quadrature_over_k(omega_m, h, n_s, sigma8):
    m = oracle.Model(omega_m=omega_m, h=h, n_s=n_s, sigma8=sigma8)
    amp = cz.sigma8_amplitude(m)
    R = 8.0

    def window(y):
        # transform of the unit-volume top-hat, written with its small-y series
        if y < 1e-3:
            return 1.0 - y * y / 10.0
        return 3.0 * (math.sin(y) - y * math.cos(y)) / y ** 3

    def integrand(k):
        return 4.0 * math.pi * k * k * float(cz.power(k, m, amp)) * window(k * R) ** 2 / (2.0 * math.pi) ** 3

    edges = np.concatenate([[1e-5], np.geomspace(1e-3, 1e3, 121)])
    total = 0.0
    for lo, hi in zip(edges[:-1], edges[1:]):
        v, _ = integrate.quad(integrand, lo, hi, epsabs=0, epsrel=1e-12, limit=400)
        total += v
    assert abs(math.sqrt(total) / sigma8 - 1) < 1e-8


def _hs_exact(m, a):
    """(M1, M2, neglected-term size) from eq. husawicki with n = 1."""
    h0 = 100.0 / C_KMS
    beta2 = h0 * h0 * m.omega_m
    r = 6.0 * (1.0 - m.omega_m) / m.omega_m            # c1/c2

    def ricci(aa):
        return _ricci(aa, m)

    # c2 from f_R(R0) = -|f_R0| with f_R = -c1/(c2 y + 1)^2, y = R/beta^2
    # (large root of |f| y0^2 c2^2 + (2|f| y0 - r) c2 + |f| = 0)
    f0 = m.fr0_abs
    y0 = ricci(1.0) / beta2
    bq = 2.0 * f0 * y0 - r
    c2 = (-bq + math.sqrt(bq * bq - 4.0 * f0 * f0 * y0 * y0)) / (2.0 * f0 * y0 * y0)
    c1 = r * c2

    def r_of_fr(fr):
        # inverse of f_R(R): c2 R/beta^2 + 1 = sqrt(c1/(-f_R))
        return beta2 * (math.sqrt(c1 / (-fr)) - 1.0) / c2

    ybar = ricci(a) / beta2
    fbar = -c1 / (c2 * ybar + 1.0) ** 2
    hstep = 1e-3 * abs(fbar)
    v = [r_of_fr(fbar + j * hstep) for j in (-2, -1, 0, 1, 2)]
    d1 = (v[0] - 8 * v[1] + 8 * v[3] - v[4]) / (12 * hstep)
    d2 = (-v[0] + 16 * v[1] - 30 * v[2] + 16 * v[3] - v[4]) / (12 * hstep * hstep)
    return d1, d2, 1.0 / (c2 * ybar)


@pytest.mark.parametrize("fr0", [1e-4, 1e-5, 1e-6])
@pytest.mark.parametrize("a", [1.0, 0.5])
def test_hu_sawicki_coefficients_are_derivatives_of_r_of_fr(fr0, a):
    m = oracle.Model(omega_m=0.3, gravity="fr_hs", fr0_abs=fr0)
    m1, m2, small = _hs_exact(m, a)
    e1 = abs(3.0 * float(cz.hs_m2(a, m)) / m1 - 1)
    e2 = abs(float(cz.hs_M2(a, m)) / m2 - 1)
    tol = 4.0 * small + 1e-6
    assert small < 3e-4
    assert e1 < tol, (e1, tol)
    assert e2 < tol, (e2, tol)


def test_background_curvature_matches_the_lcdm_form_used_by_eq_mihusawicki():
    # the factor Omega_m a^-3 + 4 Omega_L of eq. mihusawicki is R/(3 H0^2)
    m = oracle.Model(omega_m=0.3)
    h0 = 100.0 / C_KMS
    for a in (1.0, 0.5, 0.2):
        ricci = _ricci(a, m)
        assert abs(ricci / (3 * h0 * h0 * (m.omega_m / a ** 3 + 4 * m.omega_l)) - 1) < 1e-8


@pytest.mark.parametrize("a", [1.0, 0.5, 0.1])
def test_four_pi_g_rho_from_friedmann(a):
    m = oracle.Model(omega_m=0.3)
    hh = _h_of_a(a, m)
    om_a = m.omega_m / a ** 3 / (m.omega_m / a ** 3 + 1.0 - m.omega_m)
    assert abs(float(cz.four_pi_g_rho(a, m)) / (1.5 * hh * hh * om_a) - 1) < 1e-13
    assert abs(float(cz.omega_m_of_a(a, m)) / om_a - 1) < 1e-13


def test_four_pi_g_rho_from_published_constants():
    # G = 4.30091e-9 Mpc (km/s)^2 / M_sun; rho_crit,0 = 2.775366e11 h^2 M_sun/Mpc^3
    m = oracle.Model(omega_m=0.3)
    g_newton = 4.30091e-9
    rho_crit = 2.775366e11
    want = 4.0 * math.pi * g_newton * rho_crit * m.omega_m / C_KMS ** 2     # (h/Mpc)^2 at a = 1
    assert abs(float(cz.four_pi_g_rho(1.0, m)) / want - 1) < 1e-5
    assert abs(float(cz.four_pi_g_rho(0.5, m)) / (want * 8.0) - 1) < 1e-5


# ---- BBKS transfer function: expansions at both ends -------------------------
# T(q) = [ln(1 + 2.34 q)/(2.34 q)] B(q)^(-1/4), B = 1 + 3.89 q + (16.1 q)^2 +
# (5.46 q)^3 + (6.71 q)^4, q = k/Gamma, Gamma = Omega_m h.  The pins below
# expand it as power series with exact rational arithmetic -- the logarithm's
# Taylor series, series products, and a power of a series by Miller's
# recurrence (P = B^alpha  =>  B P' = alpha B' P) -- an evaluation route that
# shares nothing with the oracle's closed-form expression.  Every term of B
# enters a coefficient of order <= 4 at small q, and the two top terms enter
# the large-q expansion, so a dropped or mistyped term, a wrong exponent or a
# wrong argument fails one of them.
from fractions import Fraction as Fr

BBKS = (Fr("3.89"), Fr("16.1") ** 2, Fr("5.46") ** 3, Fr("6.71") ** 4)


def _ser_mul(a, b, n):
    return [sum(a[i] * b[k - i] for i in range(k + 1)) for k in range(n)]


def _ser_pow(b, alpha, n):
    """b[0] = 1: coefficients of b(x)^alpha by Miller's recurrence."""
    p = [Fr(1)] + [Fr(0)] * (n - 1)
    for k in range(1, n):
        p[k] = sum((alpha * j - (k - j)) * b[j] * p[k - j] for j in range(1, min(k, len(b) - 1) + 1)) / k
    return p


def _bbks_small_q_series(n):
    c = Fr("2.34")
    a = [(-c) ** k / (k + 1) for k in range(n)]                 # ln(1 + c q)/(c q)
    b = [Fr(1), *BBKS] + [Fr(0)] * n
    return _ser_mul(a, _ser_pow(b, Fr(-1, 4), n), n)


@pytest.mark.parametrize("q", [1e-3, 2e-3, 5e-3, 1e-2])
def test_bbks_matches_its_small_q_expansion(q):
    coeffs = _bbks_small_q_series(16)
    series = sum(float(cf) * q ** k for k, cf in enumerate(coeffs))
    m = oracle.Model(omega_m=0.3, h=0.7)
    t = float(cz.bbks_transfer(q * m.omega_m * m.h, m))
    # the first orders by hand: c1 = -(2.34/2 + 3.89/4)
    assert abs(float(coeffs[1]) + (1.17 + 0.9725)) < 1e-15
    assert abs(t - series) < 1e-13


@pytest.mark.parametrize("q", [1e3, 1e4, 1e5])
def test_bbks_matches_its_large_q_expansion(q):
    # T (2.34 q)(6.71 q) / ln(1 + 2.34 q) = (B/(6.71 q)^4)^(-1/4), a series in 1/q
    b0, b1, b2, b3 = Fr(1), *[BBKS[2] / BBKS[3], BBKS[1] / BBKS[3], BBKS[0] / BBKS[3]]
    d = [b0, b1, b2, b3, 1 / BBKS[3]]
    coeffs = _ser_pow(d, Fr(-1, 4), 12)
    series = sum(float(cf) * (1.0 / q) ** k for k, cf in enumerate(coeffs))
    m = oracle.Model(omega_m=0.3, h=0.7)
    t = float(cz.bbks_transfer(q * m.omega_m * m.h, m))
    got = t * (2.34 * q) * (6.71 * q) / math.log1p(2.34 * q)
    assert abs(got - series) < 1e-12


def test_bbks_depends_on_k_through_k_over_omega_m_h():
    # Gamma = Omega_m h: scaling h and k together leaves T unchanged
    k = np.geomspace(1e-4, 10.0, 41)
    base = cz.bbks_transfer(k, oracle.Model(omega_m=0.3, h=0.7))
    scaled = cz.bbks_transfer(1.37 * k, oracle.Model(omega_m=0.3, h=0.7 * 1.37))
    assert np.max(np.abs(scaled / base - 1)) < 1e-13
    assert float(cz.bbks_transfer(0.0, oracle.Model())) == 1.0
