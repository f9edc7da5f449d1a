"""Grid fields of the 2LPT pipeline: delta(k), psi1, phi_,ij, S, S(k), psi2.

Test infrastructure only (FP64 CPU oracle, torch CPU tensors so that autograd
can differentiate the chain).

Conventions
  * real fields are [n][n][n], C order (x slowest, z fastest); cell size
    L/n; particle (ix, iy, iz) sits at q = (ix, iy, iz) L/n;
  * F is the unnormalised forward DFT, F^-1 carries 1/n^3 (both from the
    oracle's own transform in ``fft``);
  * k = 2 pi m / L with m the signed DFT index; spectra keep the half
    m_z in [0, n/2];
  * mask: the DC mode and every mode on a Nyquist plane (|m_i| = n/2 for any
    axis) are zero in delta(k), S(k) and every multiplier, so that the odd
    derivative multipliers i k_i are unambiguous and every spectrum is
    Hermitian.

Steps (with the passage each follows)
  delta(k) = F[w] sqrt(P(k) n^3 / V) mask          -- the linear density field
      on a regular grid (Sec. 3, procedure); white noise w shaped by sqrt(P).
  psi1     = F^-1[ i k D1(k,a)/k^2 delta(k) ]      -- Psi = grad phi (eq.
      psigradphi), phi^(1)_,ii = -delta (first-order potential equation),
      evolved per mode by D1(k,a) (text under eq. first-displ-mg).
  phi_,ij  = F^-1[ -k_i k_j/k^2 delta(k) ]          -- second derivatives of the
      initial first-order potential; the GR spatial part (Sec. 2.4, the
      factorisation paragraph) uses the unevolved field.
  S        = sum_{i<j} (phi_,ii phi_,jj - phi_,ij^2)
           = 1/2 [phi_,ii phi_,jj - phi_,ij phi_,ji]  -- eq. second-ini.
  S(k)     = F[S] mask.
  psi2     = F^-1[ D2(k,a) (-i k/k^2) S(k) ]        -- phi^(2)_,ii = S so
      phi^(2)(k) = -S(k)/k^2, Psi2 = grad phi^(2), scaled by D2(k,a) per mode
      (Sec. 2.4, approximate factorisation).
"""
from __future__ import annotations

import math

import numpy as np
import torch

from . import cosmology as cz
from . import fft, growth
from .model import Model

PAIRS = ((0, 0), (1, 1), (2, 2), (0, 1), (0, 2), (1, 2))


def as_f64(x) -> torch.Tensor:
    if isinstance(x, torch.Tensor):
        return x.to(torch.float64)
    return torch.from_numpy(np.ascontiguousarray(x, dtype=np.float64))


def modes(n: int):
    """Signed integer mode numbers (mx, my, mz) broadcastable to [n, n, n//2+1]."""
    j = np.arange(n, dtype=np.int64)
    full = np.where(j <= (n - 1) // 2, j, j - n)        # 0, 1, .., -1 (DFT order)
    half = np.arange(n // 2 + 1, dtype=np.int64)
    return full[:, None, None], full[None, :, None], half[None, None, :]


def mask(n: int) -> np.ndarray:
    """1 on kept modes, 0 on DC and on every Nyquist plane (half spectrum)."""
    mx, my, mz = modes(n)
    h = n // 2
    keep = (np.abs(mx) != h) & (np.abs(my) != h) & (mz != h)
    keep = keep & ((mx * mx + my * my + mz * mz) != 0)
    return keep.astype(np.float64)


def kvectors(m: Model):
    """(kx, ky, kz, |k|^2, |k|) as float64 numpy arrays on the half spectrum."""
    mx, my, mz = modes(m.n)
    f = 2.0 * math.pi / m.box
    kx, ky, kz = f * mx, f * my, f * mz
    k2 = kx * kx + ky * ky + kz * kz
    return kx, ky, kz, k2, np.sqrt(k2)


def shaping(m: Model, amplitude: float | None = None) -> np.ndarray:
    """sqrt(P(|k|) n^3 / V) times the mask, on the half spectrum."""
    _, _, _, _, kk = kvectors(m)
    msk = mask(m.n)
    safe = np.where(msk > 0, kk, 1.0)
    p = cz.power(safe, m, amplitude)
    return np.sqrt(p * m.n ** 3 / m.volume) * msk


def delta_k(w, m: Model, amplitude: float | None = None) -> torch.Tensor:
    """delta(k) = F[w] sqrt(P n^3/V) mask (complex128, half spectrum)."""
    w = as_f64(w)
    return fft.rfftn(w) * torch.from_numpy(shaping(m, amplitude))


def _irfft(x: torch.Tensor, n: int) -> torch.Tensor:
    return fft.irfftn(x, s=(n, n, n))


def _inv_k2(m: Model):
    _, _, _, k2, _ = kvectors(m)
    msk = mask(m.n)
    return np.where(msk > 0, 1.0 / np.where(k2 > 0, k2, 1.0), 0.0)


def growth_on_modes(m: Model, a: float, tab=None):
    """D1(|k|,a) and D2(|k|,a) interpolated onto every half-spectrum mode."""
    if tab is None:
        tab = growth.tables(m, a)
    kn, d1, d2 = tab
    _, _, _, _, kk = kvectors(m)
    return growth.interp(kn, d1, kk, m), growth.interp(kn, d2, kk, m)


def psi1(dk: torch.Tensor, m: Model, d1_modes: np.ndarray) -> torch.Tensor:
    """First-order displacement [3][n][n][n]: F^-1[i k_i D1 / k^2 delta(k)]."""
    kv = kvectors(m)[:3]
    ik2 = _inv_k2(m)
    out = []
    for i in range(3):
        mul = torch.from_numpy(kv[i] * d1_modes * ik2) * 1j
        out.append(_irfft(mul * dk, m.n))
    return torch.stack(out)


def phi_ij(dk: torch.Tensor, m: Model, i: int, j: int) -> torch.Tensor:
    """phi_,ij = F^-1[-k_i k_j / k^2 delta(k)] (unevolved potential)."""
    kv = kvectors(m)[:3]
    mul = torch.from_numpy(-kv[i] * kv[j] * _inv_k2(m))
    return _irfft(mul * dk, m.n)


def source(dk: torch.Tensor, m: Model) -> torch.Tensor:
    """Real-space second-order source S = sum_{i<j}(phi_,ii phi_,jj - phi_,ij^2)."""
    pxx = phi_ij(dk, m, 0, 0)
    pyy = phi_ij(dk, m, 1, 1)
    pzz = phi_ij(dk, m, 2, 2)
    s = pxx * pyy + pxx * pzz + pyy * pzz
    del pxx, pyy, pzz
    for i, j in ((0, 1), (0, 2), (1, 2)):
        p = phi_ij(dk, m, i, j)
        s = s - p * p
    return s


def source_k(s: torch.Tensor, m: Model) -> torch.Tensor:
    """S(k) = F[S] with DC and Nyquist planes zeroed."""
    return fft.rfftn(s) * torch.from_numpy(mask(m.n))


def psi2(sk: torch.Tensor, m: Model, d2_modes: np.ndarray) -> torch.Tensor:
    """Second-order displacement [3][n][n][n]: F^-1[D2 (-i k_i/k^2) S(k)]."""
    kv = kvectors(m)[:3]
    ik2 = _inv_k2(m)
    out = []
    for i in range(3):
        mul = torch.from_numpy(-kv[i] * d2_modes * ik2) * 1j
        out.append(_irfft(mul * sk, m.n))
    return torch.stack(out)


def displace(w, m: Model, a: float, tab=None, amplitude: float | None = None):
    """(psi1, psi2) in Mpc/h for white noise ``w`` at scale factor ``a``."""
    d1m, d2m = growth_on_modes(m, a, tab)
    dk = delta_k(w, m, amplitude)
    p1 = psi1(dk, m, d1m)
    s = source(dk, m)
    p2 = psi2(source_k(s, m), m, d2m)
    return p1, p2


def displace_from_delta_k(dk: torch.Tensor, m: Model, a: float, tab=None):
    """Same as ``displace`` but starting from a given delta(k) (no shaping)."""
    d1m, d2m = growth_on_modes(m, a, tab)
    dk = dk * torch.from_numpy(mask(m.n))
    p1 = psi1(dk, m, d1m)
    p2 = psi2(source_k(source(dk, m), m), m, d2m)
    return p1, p2


def lagrangian_grid(m: Model) -> torch.Tensor:
    """Particle positions q [3][n][n][n] on the regular grid (eq. position)."""
    c = torch.arange(m.n, dtype=torch.float64) * (m.box / m.n)
    gx, gy, gz = torch.meshgrid(c, c, c, indexing="ij")
    return torch.stack([gx, gy, gz])


def positions(p1: torch.Tensor, p2: torch.Tensor, m: Model) -> torch.Tensor:
    """Eulerian positions x = (q + psi1 + psi2) mod L (eq. position)."""
    return torch.remainder(lagrangian_grid(m) + p1 + p2, m.box)
