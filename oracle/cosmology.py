"""Background cosmology, Hu-Sawicki f(R) coefficients, mu(k,a) and P(k).

Test infrastructure only (FP64 CPU oracle).  Units: c = 1, lengths in Mpc/h,
wavenumbers in h/Mpc, so H0 = 100 km/s/Mpc / c = 1/2997.92458 h/Mpc.

Readings taken here (the paper leaves them implicit):
  * flat background without radiation, H^2 = H0^2 (Omega_m a^-3 + Omega_L)
    (Sec. 2.3: the Hu-Sawicki model is chosen to reproduce the LCDM
    expansion history);
  * 4 pi G rho_bar(a) = 1.5 H0^2 Omega_m a^-3, the coefficient that multiplies
    mu in eq. first-displ-mg and eq. d1;
  * the power spectrum is BBKS with Gamma = Omega_m h times k^n_s, normalised
    to sigma8 with a top-hat of radius 8 Mpc/h (the paper takes its P(k)
    from the N-body initial conditions, which are not available).
"""
from __future__ import annotations

import math

import numpy as np

from .model import Model

C_KMS = 299792.458
H0 = 100.0 / C_KMS          # h/Mpc


def e2(a, m: Model):
    """H^2/H0^2 for a flat matter + Lambda background."""
    return m.omega_m * np.power(a, -3.0) + m.omega_l


def omega_m_of_a(a, m: Model):
    """Omega_m(a) = Omega_m a^-3 / E^2(a)."""
    return m.omega_m * np.power(a, -3.0) / e2(a, m)


def four_pi_g_rho(a, m: Model):
    """4 pi G rho_bar(a) = (3/2) H0^2 Omega_m a^-3, in (h/Mpc)^2."""
    return 1.5 * H0 * H0 * m.omega_m * np.power(a, -3.0)


def hs_m2(a, m: Model):
    """Scalar-field mass squared m^2(a) = M1(a)/3 (eq. mihusawicki, n = 1).

    M1 = (3/2) (H0^2/|f_R0|) (Omega_m a^-3 + 4 Omega_L)^3 / (Omega_m + 4 Omega_L)^2,
    and the text under eq. first-displ-mg relates M1 = 3 m^2.
    """
    x = m.omega_m * np.power(a, -3.0) + 4.0 * m.omega_l
    x0 = m.omega_m + 4.0 * m.omega_l
    return 0.5 * (H0 * H0 / m.fr0_abs) * x ** 3 / x0 ** 2


def hs_M2(a, m: Model):
    """Second expansion coefficient M2(a) (eq. mihusawicki, n = 1).

    M2 = (9/4) (H0^2/|f_R0|^2) (Omega_m a^-3 + 4 Omega_L)^5 / (Omega_m + 4 Omega_L)^4.
    """
    x = m.omega_m * np.power(a, -3.0) + 4.0 * m.omega_l
    x0 = m.omega_m + 4.0 * m.omega_l
    return 2.25 * (H0 * H0 / (m.fr0_abs * m.fr0_abs)) * x ** 5 / x0 ** 4


def mu(k, a, m: Model):
    """Scale-dependent Poisson factor mu(k,a) (Sec. 2.4, below eq. first-displ-mg).

    GR: 1.  Hu-Sawicki: 1 + (1/3) (k^2/a^2) / (k^2/a^2 + m^2(a)).
    mu_const (a test model that is not in the paper): the constant m.mu_const.
    """
    k = np.asarray(k, dtype=np.float64)
    if m.gravity == "gr":
        return np.ones_like(k)
    if m.gravity == "mu_const":
        return np.full_like(k, m.mu_const)
    q = k * k / (a * a)
    return 1.0 + (1.0 / 3.0) * q / (q + hs_m2(a, m))


def big_pi(k, a, m: Model):
    """Pi(k,a) = k^2/a^2 + m^2(a) (defined after eq. s4).  Hu-Sawicki only."""
    k = np.asarray(k, dtype=np.float64)
    return k * k / (a * a) + hs_m2(a, m)


def bbks_transfer(k, m: Model):
    """BBKS (Bardeen, Bond, Kaiser & Szalay 1986) transfer function, q = k/Gamma,
    Gamma = Omega_m h.  Pinned to its power-series expansions at small and at
    large q (exact rational series arithmetic in the tests) and to its
    dependence on k through k/Gamma."""
    k = np.asarray(k, dtype=np.float64)
    q = k / (m.omega_m * m.h)
    x = 2.34 * q
    poly = 1.0 + 3.89 * q + (16.1 * q) ** 2 + (5.46 * q) ** 3 + (6.71 * q) ** 4
    with np.errstate(divide="ignore", invalid="ignore"):
        t = np.log1p(x) / x * poly ** -0.25
    return np.where(q > 0, t, 1.0)


def tophat_window(x):
    """Fourier transform of a unit top-hat sphere, 3 (sin x - x cos x) / x^3."""
    x = np.asarray(x, dtype=np.float64)
    return 3.0 * (np.sin(x) - x * np.cos(x)) / x ** 3


def sigma8_amplitude(m: Model, intervals: int = 1 << 16) -> float:
    """Amplitude A such that P(k) = A k^n_s T^2(k) has sigma(8 Mpc/h) = sigma8.

    Pinned by an adaptive quadrature of int d^3k/(2 pi)^3 P W^2 over k.

    sigma^2 = (1/2 pi^2) Int k^3 P(k) W^2(8k) dln k, composite Simpson on
    ln k in [ln 1e-5, ln 1e3] with ``intervals`` (even) sub-intervals.
    """
    lo, hi = math.log(1e-5), math.log(1e3)
    x = np.linspace(lo, hi, intervals + 1)
    k = np.exp(x)
    f = k ** 3 * k ** m.n_s * bbks_transfer(k, m) ** 2 * tophat_window(8.0 * k) ** 2
    f /= 2.0 * math.pi ** 2
    h = (hi - lo) / intervals
    s = f[0] + f[-1] + 4.0 * f[1:-1:2].sum() + 2.0 * f[2:-1:2].sum()
    return m.sigma8 ** 2 / (s * h / 3.0)


def power(k, m: Model, amplitude: float | None = None):
    """Linear matter power spectrum at a = 1 in (Mpc/h)^3."""
    if amplitude is None:
        amplitude = sigma8_amplitude(m)
    k = np.asarray(k, dtype=np.float64)
    return amplitude * k ** m.n_s * bbks_transfer(k, m) ** 2
