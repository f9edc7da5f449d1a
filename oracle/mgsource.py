"""Full modified-gravity source S1+S2+S3+S4, its ratio to GR, and the triangle choice.

Test infrastructure only (FP64 CPU oracle).

The paper writes the right-hand side of the 2LPT equation in f(R) as four
terms built from Fourier transforms of local products (eq. full and eqs.
s1-s4), computes them on a grid from a density field evolved with D1(k,a),
divides by the GR source of the same field, bins the ratio in k (mean and
scatter) and compares the bin means with the analytic ratio of candidate
triangle configurations (Sec. 3, the procedure and triangle-comparison
paragraphs).

Readings taken here:
  * eq. s1 as printed has no GR limit: with mu = 1, S1 + S2 does not reduce
    to the GR source.  The convolution form of eq. displ2 with the kernel of
    eq. full-d2 requires S1 = G { F[phi_ij F^-1[mu F phi_ji]] - mu(k) F[phi_ij phi_ji] }
    (G = 4 pi G rho_bar); the extra term is the mu(k) c^2 piece of the
    kernel.  This is what is computed, and tests pin the sum S1..S4 to the
    brute-force triangle sum of the eq. full-d2 kernel.
  * phi^(1), delta^(1) inside S1..S4 are evolved by D1(k,a) (text after eq.
    s4); S_GR = -(G/2) D1_GR(a)^2 F[(tr phi)^2 - phi_ij phi_ji] from the
    unevolved potential, D1_GR normalised to 1 at a = 1.
  * the ratio of the source to its LCDM counterpart (Sec. 3, the procedure
    paragraph) is taken, for complex values, as Re(S_MG conj(S_GR)) / |S_GR|^2
    per mode; modes with S_GR = 0 are left out.
  * triangle choice: weighted least squares of the bin means against the
    analytic ratio R_T(k) = D1(k1) D1(k2) B(k,k1,k2) / (D1_GR^2 (1 - c^2)),
    counts as weights, bins with mean k <= 0.4 h/Mpc.  The squeezed triangle
    is taken as k1/k2 = 1e-3 at 90 degrees.
"""
from __future__ import annotations

import math

import numpy as np
import torch

from . import cosmology as cz
from . import fft, fields, growth, spectrum
from .model import Model

CANDIDATES = (
    ("T1", 1.0, 90.0, False),
    ("T2", 1.0, 80.0, False),
    ("iso70", 1.0, 70.0, False),
    ("equilateral", 1.0, 60.0, False),
    ("squeezed", 1e-3, 90.0, False),
    ("r2_80", 2.0, 80.0, False),
    ("r2_70", 2.0, 70.0, False),
    ("winther", 1.0, 90.0, True),
)


def d1_gr(a: float, m: Model) -> float:
    """Normalised GR linear growth D1_GR(a) (k-independent)."""
    g = m.with_(gravity="gr", factorisation="eds")
    d, _ = growth.solve(np.zeros(1), a, g, with_d2=False)
    return float(d[0]) / growth.normalisation(g)


def _irfft(x, n):
    return fft.irfftn(x, s=(n, n, n))


def _rfft(x):
    return fft.rfftn(x)


def full_source(w, m: Model, a: float, tab=None):
    """S_MG(k) = S1 + S2 + S3 + S4 on the half spectrum (eqs. full, s1-s4)."""
    return full_source_dk(fields.delta_k(w, m), m, a, tab)


def full_source_dk(dk: torch.Tensor, m: Model, a: float, tab=None):
    """S1 + S2 + S3 + S4 from a given unevolved delta(k) (half spectrum)."""
    n = m.n
    d1m, _ = fields.growth_on_modes(m, a, tab)
    da = dk * torch.from_numpy(d1m * fields.mask(n))
    kx, ky, kz, k2, kk = fields.kvectors(m)
    kv = (kx, ky, kz)
    msk = fields.mask(n)
    ik2 = np.where(msk > 0, 1.0 / np.where(k2 > 0, k2, 1.0), 0.0)
    mu_k = torch.from_numpy(np.broadcast_to(cz.mu(kk, a, m), msk.shape).copy())
    g = float(cz.four_pi_g_rho(a, m))

    r1 = torch.zeros((n, n, n), dtype=torch.float64)
    r2 = torch.zeros_like(r1)
    tr = torch.zeros_like(r1)
    for i, j in fields.PAIRS:
        mult = 1.0 if i == j else 2.0
        base = -kv[i] * kv[j] * ik2
        pa = _irfft(torch.from_numpy(base) * da, n)
        pm = _irfft(torch.from_numpy(base) * mu_k * da, n)
        r1 = r1 + mult * pa * pm
        r2 = r2 + mult * pa * pa
        if i == j:
            tr = tr + pa
    f_r2 = _rfft(r2)
    s = g * (_rfft(r1) - mu_k * f_r2)                         # S1 (corrected)
    s = s - 0.5 * g * mu_k * (_rfft(tr * tr) - f_r2)          # S2

    if m.gravity == "fr_hs":
        ms = float(cz.hs_m2(a, m))
        big_m2 = float(cz.hs_M2(a, m))
        pi_k = cz.big_pi(kk, a, m)
        ipi = torch.from_numpy(np.broadcast_to(1.0 / pi_k, msk.shape).copy())
        chi = _irfft(ipi * da, n)
        pre3 = (2.0 * g / 3.0) ** 2 * (big_m2 / 12.0) * (kk * kk / (a * a)) / pi_k
        s = s + torch.from_numpy(np.broadcast_to(pre3, msk.shape).copy()) * _rfft(chi * chi)   # S3
        r5 = torch.zeros_like(r1)
        for i, j in fields.PAIRS:
            mult = 1.0 if i == j else 2.0
            pa = _irfft(torch.from_numpy(-kv[i] * kv[j] * ik2) * da, n)
            cij = _irfft(torch.from_numpy(-kv[i] * kv[j]) * ipi * da, n)
            r5 = r5 + 2.0 * mult * pa * cij
        for j in range(3):
            piij = _irfft(torch.from_numpy(kv[j]) * da * (-1j), n)
            cj = _irfft(torch.from_numpy(kv[j]) * ipi * da * 1j, n)
            r5 = r5 + piij * cj
        pre4 = -(2.0 * g / 3.0) * (ms / (2.0 * a * a)) / pi_k
        s = s + torch.from_numpy(np.broadcast_to(pre4, msk.shape).copy()) * _rfft(r5)          # S4
    return s * torch.from_numpy(msk)


def gr_source(w, m: Model, a: float):
    """S_GR(k) = -(G/2) D1_GR(a)^2 F[(tr phi)^2 - phi_ij phi_ji] (unevolved phi)."""
    return gr_source_dk(fields.delta_k(w, m), m, a)


def gr_source_dk(dk: torch.Tensor, m: Model, a: float):
    """S_GR(k) from a given unevolved delta(k) (half spectrum)."""
    g = float(cz.four_pi_g_rho(a, m))
    dk = dk * torch.from_numpy(fields.mask(m.n))
    sk = fields.source_k(fields.source(dk, m), m)
    return -g * d1_gr(a, m) ** 2 * sk


def ratio_modes(s_mg: torch.Tensor, s_gr: torch.Tensor):
    """(q, keep) with q = Re(S_MG conj S_GR)/|S_GR|^2 per mode; keep where S_GR != 0."""
    num = (s_mg * s_gr.conj()).real.numpy()
    den = (s_gr.abs() ** 2).numpy()
    keep = den > 0
    q = np.where(keep, num / np.where(keep, den, 1.0), 0.0)
    return q, keep


def source_ratio(w, m: Model, a: float, nbins: int, tab=None):
    """Binned (k_mean, count, mean, std) of S_MG/S_GR over the kept modes."""
    q, keep = ratio_modes(full_source(w, m, a, tab), gr_source(w, m, a))
    kmean, cnt, mean, std = _bin_kept(q, keep, m, nbins)
    return kmean, cnt, mean, std


def _bin_kept(q, keep, m: Model, nbins: int):
    b, wgt = spectrum.shell_index(m.n, nbins)
    mx, my, mz = fields.modes(m.n)
    kk = (2.0 * math.pi / m.box) * np.sqrt((mx * mx + my * my + mz * mz).astype(np.float64))
    kk = np.broadcast_to(kk, b.shape)
    sel = (b >= 0) & keep
    bs, ws = b[sel], wgt[sel].astype(np.float64)
    qs, ks = q[sel], kk[sel]
    cnt = np.bincount(bs, weights=ws, minlength=nbins)
    sk = np.bincount(bs, weights=ws * ks, minlength=nbins)
    sq = np.bincount(bs, weights=ws * qs, minlength=nbins)
    sq2 = np.bincount(bs, weights=ws * qs * qs, minlength=nbins)
    nz = cnt > 0
    safe = np.where(nz, cnt, 1.0)
    mean = np.where(nz, sq / safe, 0.0)
    std = np.sqrt(np.maximum(np.where(nz, sq2 / safe - mean * mean, 0.0), 0.0))
    return np.where(nz, sk / safe, 0.0), cnt, mean, std


def triangle_ratio(k, m: Model, a: float, ratio: float, theta_deg: float,
                   winther: bool = False, tab=None):
    """Analytic MG/GR source ratio R_T(k,a) of one triangle configuration."""
    if tab is None:
        tab = growth.tables(m.with_(factorisation="eds"), a)
    kn, d1, _ = tab
    k = np.asarray(k, dtype=np.float64)
    c = growth.cos_deg(theta_deg)
    k1, k2 = growth.triangle_sides(k, ratio, c)
    if winther:
        dd = growth.interp(kn, d1, k, m) ** 2
    else:
        dd = growth.interp(kn, d1, k1, m) * growth.interp(kn, d1, k2, m)
    b = growth.source_brace(k, k1, k2, c, a, m)
    return dd * b / (d1_gr(a, m) ** 2 * (1.0 - c * c))


def choose_triangle(kmean, cnt, mean, m: Model, a: float, kcut: float = 0.4, tab=None, metric: str = "l2"):
    """Name of the candidate with the smallest misfit over the populated
    shells with 0 < k <= kcut, and every candidate's misfit.

    metric "l2" (the reading taken for the choice): count-weighted squared
    misfit sum_b N_b (mean_b - R_T(k_b))^2; "maxrel" (a second reading, for
    comparison): max_b |mean_b / R_T(k_b) - 1|.
    """
    sel = (cnt > 0) & (kmean <= kcut) & (kmean > 0)
    best, best_cost, costs = None, math.inf, {}
    for name, r, th, win in CANDIDATES:
        rt = triangle_ratio(kmean[sel], m, a, r, th, win, tab)
        if metric == "maxrel":
            cost = float(np.max(np.abs(mean[sel] / rt - 1.0)))
        else:
            cost = float(np.sum(cnt[sel] * (mean[sel] - rt) ** 2))
        costs[name] = cost
        if cost < best_cost:
            best, best_cost = name, cost
    return best, costs


def direct_triangle_sum(dk: np.ndarray, m: Model, a: float, tab=None):
    """Brute-force -(G/2)(1/n^3) sum_{k1+k2=k} D1 D1 B(k,k1,k2) delta1 delta2.

    The O(n^6) convolution of eq. displ2 with the braced kernel of eq. full-d2
    (without the GR normalisation), over a full complex spectrum ``dk``
    [n][n][n].  Only for tiny band-limited grids (the result is exact when no
    k1 + k2 wraps around).  The loop runs over k1; all k2 are handled at once.
    """
    n = m.n
    if tab is None:
        tab = growth.tables(m.with_(factorisation="eds"), a)
    kn, d1, _ = tab
    f = 2.0 * math.pi / m.box
    idx = fields.modes(n)[0].reshape(-1)
    g = float(cz.four_pi_g_rho(a, m))
    pos = [(i, j, l) for i in range(n) for j in range(n) for l in range(n)
           if dk[i, j, l] != 0 and (i, j, l) != (0, 0, 0)]
    pos = np.array(pos, dtype=np.int64)
    vec = f * idx[pos].astype(np.float64)                 # [M][3] wavevectors
    kmag = np.sqrt(np.sum(vec * vec, axis=1))
    amp = dk[pos[:, 0], pos[:, 1], pos[:, 2]]
    d1v = growth.interp(kn, d1, kmag, m)
    out = np.zeros((n, n, n), dtype=np.complex128)
    for p in range(len(pos)):
        v = vec[p][None, :] + vec                         # k = k1 + k2 for all k2
        kk = np.sqrt(np.sum(v * v, axis=1))
        ok = kk > 0.0
        c = (vec @ vec[p])[ok] / (kmag[p] * kmag[ok])
        b = growth.source_brace(kk[ok], np.full(int(ok.sum()), kmag[p]), kmag[ok], c, a, m)
        contrib = d1v[p] * d1v[ok] * b * amp[p] * amp[ok]
        tgt = (pos[p][None, :] + pos[ok]) % n
        np.add.at(out, (tgt[:, 0], tgt[:, 1], tgt[:, 2]), contrib)
    return -0.5 * g * out / n ** 3
