"""Shell binning of a per-mode quantity in |k| (oracle side).

Test infrastructure only (FP64 CPU oracle).

The paper bins the source-term ratio in a grid of k values and reports the
mean and the scatter in each bin (Sec. 3, the procedure paragraph and the
discussion of the source-term figure).  Readings taken here:
  * nbins equal shells of width dk = k_Nyq / nbins, k_Nyq = pi n / L;
  * shell index b = floor(|k| / dk), computed exactly in integers from the
    integer mode numbers: b = isqrt(floor(|m|^2 nbins^2 / (n/2)^2));
  * the DC mode and modes with b >= nbins are left out (so every Nyquist
    plane is left out);
  * each half-spectrum mode stands for itself and its conjugate partner:
    weight 2 for 0 < m_z < n/2, weight 1 on the m_z = 0 plane;
  * mean = sum(w q) / sum(w); std = sqrt(max(0, sum(w q^2)/sum(w) - mean^2))
    (population scatter); k_mean = sum(w |k|)/sum(w); an empty bin reports
    zeros.
"""
from __future__ import annotations

import math

import numpy as np
import torch

from . import fft
from .fields import modes
from .model import Model


def isqrt_array(v: np.ndarray) -> np.ndarray:
    """Exact floor(sqrt(v)) for non-negative int64 arrays."""
    r = np.floor(np.sqrt(v.astype(np.float64))).astype(np.int64)
    r = np.where(r * r > v, r - 1, r)
    r = np.where((r + 1) * (r + 1) <= v, r + 1, r)
    return r


def shell_index(n: int, nbins: int):
    """(bin index, weight) on the half spectrum; -1 marks modes left out."""
    mx, my, mz = modes(n)
    m2 = (mx * mx + my * my + mz * mz).astype(np.int64)
    h = n // 2
    b = isqrt_array((m2 * nbins * nbins) // (h * h))
    w = np.where(mz == 0, 1, 2).astype(np.int64) * np.ones_like(m2)
    b = np.where((m2 == 0) | (b >= nbins), -1, b)
    return b, w


def bin_shells(q: np.ndarray, m: Model, nbins: int):
    """(k_mean, count, mean, std) per shell for per-mode values ``q``."""
    q = np.asarray(q, dtype=np.float64)
    b, w = shell_index(m.n, nbins)
    mx, my, mz = modes(m.n)
    kk = (2.0 * math.pi / m.box) * np.sqrt((mx * mx + my * my + mz * mz).astype(np.float64))
    kk = np.broadcast_to(kk, b.shape)
    sel = b >= 0
    bs, ws = b[sel], w[sel].astype(np.float64)
    qs, ks = np.broadcast_to(q, b.shape)[sel], kk[sel]
    cnt = np.bincount(bs, weights=ws, minlength=nbins)
    sk = np.bincount(bs, weights=ws * ks, minlength=nbins)
    sq = np.bincount(bs, weights=ws * qs, minlength=nbins)
    sq2 = np.bincount(bs, weights=ws * qs * qs, minlength=nbins)
    nz = cnt > 0
    safe = np.where(nz, cnt, 1.0)
    kmean = np.where(nz, sk / safe, 0.0)
    mean = np.where(nz, sq / safe, 0.0)
    var = np.where(nz, sq2 / safe - mean * mean, 0.0)
    std = np.sqrt(np.maximum(var, 0.0))
    return kmean, cnt, mean, std


def source_power(sk, m: Model, nbins: int):
    """Shell-averaged power of the source, q = V |S(k)/n^3|^2."""
    s = sk.detach().numpy() if hasattr(sk, "detach") else np.asarray(sk)
    q = m.volume * np.abs(s / m.n ** 3) ** 2
    return bin_shells(q, m, nbins)


def cic_window(m: Model) -> np.ndarray:
    """Fourier window of cloud-in-cell assignment on the half spectrum:
    W(m) = prod_i sinc^2(pi m_i / n), the transform of the linear (triangle)
    kernel along each axis (sinc x = sin x / x)."""
    mx, my, mz = modes(m.n)
    return (np.sinc(mx / m.n) * np.sinc(my / m.n) * np.sinc(mz / m.n)) ** 2


def matter_power(delta, m: Model, nbins: int, deconvolve: bool = False):
    """Shell-averaged power of a real density contrast on the grid,
    q = V |F[delta]/n^3|^2, optionally divided by the CIC window squared."""
    d = delta.detach().numpy() if hasattr(delta, "detach") else np.asarray(delta)
    dk = fft.rfftn(torch.from_numpy(np.asarray(d, dtype=np.float64))).numpy()
    return _power_of(dk, m, nbins, deconvolve)


def _power_of(dk: np.ndarray, m: Model, nbins: int, deconvolve: bool):
    q = m.volume * np.abs(dk / m.n ** 3) ** 2
    if deconvolve:
        q = q / cic_window(m) ** 2
    return bin_shells(q, m, nbins)


def interlaced_density_k(disp, m: Model) -> np.ndarray:
    """F[delta] with interlacing (the alias reduction of grid mass assignment
    used for the matter power the paper compares, Sec. 4): the particles are
    painted twice, the second time moved by half a cell along every axis;
    that move multiplies the second transform by exp(-i pi (m_x+m_y+m_z)/n)
    for the modes inside the Nyquist cube, so it is multiplied back, and the
    two transforms are averaged.  The alias images whose index sum is odd
    enter the two with opposite signs and cancel."""
    from . import cic
    d = torch.as_tensor(disp, dtype=torch.float64)
    d1 = cic.paint(d, m).numpy()
    d2 = cic.paint(d + m.box / (2 * m.n), m).numpy()
    mx, my, mz = modes(m.n)
    phase = np.exp(1j * np.pi * (mx + my + mz) / m.n)
    f1 = fft.rfftn(torch.from_numpy(d1)).numpy()
    f2 = fft.rfftn(torch.from_numpy(d2)).numpy()
    return 0.5 * (f1 + f2 * phase)


def matter_power_interlaced(disp, m: Model, nbins: int, deconvolve: bool = False):
    """matter_power of the interlaced CIC density of particles displaced by
    ``disp`` [3][n][n][n] (Mpc/h) from the grid points."""
    return _power_of(interlaced_density_k(disp, m), m, nbins, deconvolve)
