"""Scale-dependent growth factors D1(k,a) and D2(k,a) (oracle side).

Test infrastructure only (FP64 CPU oracle).

D1 solves eq. d1 for each k, with mu(k,a) inside the operator; D2 solves
eq. full-d2 for one triangle (k, k1, k2) with |k1 + k2| = k, which is how the
paper obtains its k-dependent D2(k,a) (Sec. 3, end of the triangle
comparison: the orthogonal isosceles triangle T1 is adopted).  Each k is
solved independently and the table is interpolated in k (Sec. 2.4, text
under eq. d1).

Readings (the printed equations are ambiguous here):
  * eq. motion brackets d/da inside the friction term and eq. d1 writes
    a^2 H^2 (T - 4 pi G rho mu); the dimensionally consistent operator is
    a^2 H^2 T - 4 pi G rho mu with T = d2/da2 + (3/a + H'/H) d/da.  In
    x = ln a, dividing by H^2:
        D'' + (2 - 1.5 Omega_m(a)) D' - 1.5 Omega_m(a) mu(k,a) D = RHS.
  * eq. full-d2's right-hand side has the opposite sign to the GR D2
    equation and is not divided by the GR angular factor.  The GR limit fixes
    both: RHS = -1.5 Omega_m(a) D1(k1) D1(k2) B(k,k1,k2,a) / (1 - cos^2 theta),
    where B is the braced expression of eq. full-d2.  With mu = 1 this is the
    GR equation and gives D2 = -3/7 D1^2 in Einstein-de Sitter.
  * Runge-Kutta flavour and step count are not given: classical RK4 in ln a
    with a fixed number of equal steps from a_init.
  * initial conditions: the EdS growing mode, D1 = a_init, dD1/dln a = a_init
    (Sec. 2.4); for D2, D2 = -3/7 a_init^2, dD2/dln a = -6/7 a_init^2.  The
    constant-mu test model (not in the paper) starts on its own EdS power law.
  * normalisation D1(k -> 0, a = 1) = 1 (Sec. 2.4), obtained by integrating
    the k = 0 equation to a = 1; D2 is divided by the square of that number.
  * nodes: nk log-spaced k from kmin to kmax inclusive; interpolation linear in
    ln k; clamped outside the node range.
  * an angle of exactly 90 degrees uses cos = 0 exactly.
"""
from __future__ import annotations

import math

import numpy as np

from . import cosmology as cz
from .model import Model


def cos_deg(theta_deg: float) -> float:
    """cos(theta) with exact zero at 90 degrees."""
    if theta_deg == 90.0:
        return 0.0
    return math.cos(math.radians(theta_deg))


def triangle_sides(k, ratio: float, cos_t: float):
    """Sides k1 = r k2 and k2 such that |k1 + k2| = k at angle theta between them."""
    k = np.asarray(k, dtype=np.float64)
    k2 = k / math.sqrt(1.0 + ratio * ratio + 2.0 * ratio * cos_t)
    return ratio * k2, k2


def source_brace(k, k1, k2, cos_t: float, a: float, m: Model):
    """The braced factor B(k, k1, k2, a) of eq. full-d2.

    B = mu(k) - c^2 [mu(k1) + mu(k2) - mu(k)]
        + m^2/Pi(k) [ 2 c^2 (mu(k1) + mu(k2) - 2) + (k1.k2/k1^2)(mu(k1) - 1)
                      + (k1.k2/k2^2)(mu(k2) - 1) ]
        - (2/27) 4piG rho (k^2/a^2) M2 / (Pi(k) Pi(k1) Pi(k2)),
    with c = cos(theta) (a scalar, or an array matching k) and k1.k2 = k1 k2 c.
    In GR and for the constant-mu
    test model there is no scalar mass, and the last two terms are absent.
    """
    c2 = cos_t * cos_t
    mk, m1, m2 = cz.mu(k, a, m), cz.mu(k1, a, m), cz.mu(k2, a, m)
    b = mk - c2 * (m1 + m2 - mk)
    if m.gravity == "fr_hs":
        ms = cz.hs_m2(a, m)
        pk, p1, p2 = cz.big_pi(k, a, m), cz.big_pi(k1, a, m), cz.big_pi(k2, a, m)
        dot = k1 * k2 * cos_t
        bracket = (2.0 * c2 * (m1 + m2 - 2.0) + dot / (k1 * k1) * (m1 - 1.0)
                   + dot / (k2 * k2) * (m2 - 1.0))
        b = b + ms / pk * bracket
        b = b - (2.0 / 27.0) * cz.four_pi_g_rho(a, m) * (k * k / (a * a)) * cz.hs_M2(a, m) / (pk * p1 * p2)
    return b


def _initial_state(m: Model, n: int):
    """EdS growing modes at a_init for (D1(k), D1(k1), D1(k2), D2) and slopes."""
    ai = m.a_init
    if m.gravity == "mu_const":
        # EdS with constant mu: D1 = a^p, p^2 + p/2 - 1.5 mu = 0; D2 = c a^{2p}.
        mu0 = m.mu_const
        p = (-0.5 + math.sqrt(0.25 + 6.0 * mu0)) / 2.0
        c = -1.5 * mu0 / (4.0 * p * p + p - 1.5 * mu0)
        d1, s1 = ai ** p, p * ai ** p
        d2, s2 = c * ai ** (2 * p), 2.0 * p * c * ai ** (2 * p)
    else:
        d1, s1 = ai, ai
        d2, s2 = -3.0 / 7.0 * ai * ai, -6.0 / 7.0 * ai * ai
    y = np.empty((8, n))
    y[0] = d1; y[1] = s1      # D1(k)
    y[2] = d1; y[3] = s1      # D1(k1)
    y[4] = d1; y[5] = s1      # D1(k2)
    y[6] = d2; y[7] = s2      # D2(k)
    return y


def _rhs(x, y, k, k1, k2, cos_t, bgr, winther, m: Model, with_d2: bool):
    a = math.exp(x)
    om = float(cz.omega_m_of_a(a, m))
    fr = 2.0 - 1.5 * om
    g = 1.5 * om
    dy = np.empty_like(y)
    mk = cz.mu(k, a, m)
    dy[0] = y[1]
    dy[1] = -fr * y[1] + g * mk * y[0]
    if with_d2:
        dy[2] = y[3]
        dy[3] = -fr * y[3] + g * cz.mu(k1, a, m) * y[2]
        dy[4] = y[5]
        dy[5] = -fr * y[5] + g * cz.mu(k2, a, m) * y[4]
        src = y[0] * y[0] if winther else y[2] * y[4]
        b = source_brace(k, k1, k2, cos_t, a, m)
        dy[6] = y[7]
        dy[7] = -fr * y[7] + g * mk * y[6] - g * src * b / bgr
    else:
        dy[2:] = 0.0
    return dy


def solve(k, a: float, m: Model, ratio: float = 1.0, theta_deg: float = 90.0,
          winther: bool = False, with_d2: bool = True, steps: int | None = None):
    """Unnormalised D1(k,a) and D2(k,a) at the wavenumbers ``k`` (array).

    Classical RK4 in x = ln a from ln a_init to ln a with ``steps`` equal steps.
    """
    k = np.atleast_1d(np.asarray(k, dtype=np.float64))
    steps = m.ode_steps if steps is None else steps
    cos_t = cos_deg(theta_deg)
    k1, k2 = triangle_sides(k, ratio, cos_t)
    bgr = 1.0 - cos_t * cos_t
    y = _initial_state(m, k.size)
    x0, x1 = math.log(m.a_init), math.log(a)
    h = (x1 - x0) / steps
    for s in range(steps):
        x = x0 + s * h
        f1 = _rhs(x, y, k, k1, k2, cos_t, bgr, winther, m, with_d2)
        f2 = _rhs(x + 0.5 * h, y + 0.5 * h * f1, k, k1, k2, cos_t, bgr, winther, m, with_d2)
        f3 = _rhs(x + 0.5 * h, y + 0.5 * h * f2, k, k1, k2, cos_t, bgr, winther, m, with_d2)
        f4 = _rhs(x + h, y + h * f3, k, k1, k2, cos_t, bgr, winther, m, with_d2)
        y = y + (h / 6.0) * (f1 + 2.0 * f2 + 2.0 * f3 + f4)
    return y[0].copy(), y[6].copy()


def normalisation(m: Model) -> float:
    """D1(k = 0, a = 1) from the same integrator (Sec. 2.4 normalisation)."""
    d1, _ = solve(np.zeros(1), 1.0, m, with_d2=False)
    return float(d1[0])


def nodes(m: Model) -> np.ndarray:
    """nk log-spaced wavenumbers from kmin to kmax inclusive."""
    lo, hi = math.log(m.kmin), math.log(m.kmax)
    b = np.arange(m.nk, dtype=np.float64)
    return np.exp(lo + (hi - lo) * b / (m.nk - 1))


def tables(m: Model, a: float):
    """Growth tables on the k nodes: (k, D1(k,a), D2(k,a)), normalised.

    The D2 column follows ``m.factorisation``:
      eds      -- D2 = -3/7 D1^2;
      t1       -- eq. full-d2 with k1 = k2, theta = 90 degrees (T1);
      triangle -- eq. full-d2 with k1/k2 = tri_ratio at tri_theta_deg;
      winther  -- T1 geometry with D1(k)^2 in place of D1(k1) D1(k2);
      bouchet  -- D2 = -3/7 D1^2 Omega_m(a)^(-1/143) (eq. lcdm-fit).
    """
    k = nodes(m)
    norm = normalisation(m)
    f = m.factorisation
    if f == "t1":
        d1, d2 = solve(k, a, m, 1.0, 90.0)
    elif f == "triangle":
        d1, d2 = solve(k, a, m, m.tri_ratio, m.tri_theta_deg)
    elif f == "winther":
        d1, d2 = solve(k, a, m, 1.0, 90.0, winther=True)
    else:
        d1, _ = solve(k, a, m, with_d2=False)
        d2 = None
    d1 = d1 / norm
    if f == "eds":
        d2 = -3.0 / 7.0 * d1 * d1
    elif f == "bouchet":
        d2 = -3.0 / 7.0 * d1 * d1 * float(cz.omega_m_of_a(a, m)) ** (-1.0 / 143.0)
    else:
        d2 = d2 / (norm * norm)
    return k, d1, d2


def interp(kn: np.ndarray, table: np.ndarray, k, m: Model):
    """Linear interpolation in ln k on the node table, clamped at both ends."""
    k = np.asarray(k, dtype=np.float64)
    lo, hi = math.log(m.kmin), math.log(m.kmax)
    with np.errstate(divide="ignore"):
        u = (np.log(k) - lo) / (hi - lo) * (m.nk - 1)
    u = np.clip(u, 0.0, m.nk - 1.0)
    i = np.minimum(np.floor(u).astype(np.int64), m.nk - 2)
    t = u - i
    return table[i] + t * (table[i + 1] - table[i])
