"""The oracle's own discrete Fourier transform (mixed-radix Cooley-Tukey).

Test infrastructure only (FP64 CPU oracle).  Every F and F^-1 of the oracle
goes through this module; it calls no FFT library.  Written in torch tensor
operations (reshape, transpose, elementwise products and small dense matrix
products) so that autograd differentiates through it.

Definition (the convention every other oracle module uses):
    F[x](k)    = sum_j x(j) exp(-2 pi i j k / n)        (unnormalised)
    F^-1[X](j) = (1/n) sum_k X(k) exp(+2 pi i j k / n)
applied along each axis of a 3D array.  The real transforms keep the half
spectrum m_z in [0, n/2] along the last axis.

Method.  A length n = n1 n2 splits by the Cooley-Tukey index map: input
index j = n2 j1 + j2, output index k = k1 + n1 k2, so that
    X(k1 + n1 k2) = sum_j2 W_n2^(j2 k2) [ W_n^(j2 k1) sum_j1 W_n1^(j1 k1) x(n2 j1 + j2) ],
W_m = exp(-/+ 2 pi i / m): n2 transforms of length n1, a twiddle product,
n1 transforms of length n2.  Lengths of at most ``DIRECT`` points, and prime
lengths, are evaluated directly from the definition as a product with the
n x n matrix W^(j k).  Any n > 0 is accepted; the grids used here factor
into 2, 3, 5 and 7.
"""
from __future__ import annotations

import math
from functools import lru_cache

import torch

DIRECT = 32


@lru_cache(maxsize=None)
def _dft_matrix(n: int, sign: int) -> torch.Tensor:
    """[k][j] = exp(sign 2 pi i j k / n), with j k reduced mod n before the
    angle is formed (exact symmetry, no growth of the argument)."""
    jk = (torch.arange(n, dtype=torch.int64)[:, None] * torch.arange(n, dtype=torch.int64)[None, :]) % n
    ang = (sign * 2.0 * math.pi / n) * jk.to(torch.float64)
    return torch.polar(torch.ones_like(ang), ang)


@lru_cache(maxsize=None)
def _twiddle(n1: int, n2: int, sign: int) -> torch.Tensor:
    """[j2][k1] = exp(sign 2 pi i j2 k1 / (n1 n2))."""
    n = n1 * n2
    jk = (torch.arange(n2, dtype=torch.int64)[:, None] * torch.arange(n1, dtype=torch.int64)[None, :]) % n
    ang = (sign * 2.0 * math.pi / n) * jk.to(torch.float64)
    return torch.polar(torch.ones_like(ang), ang)


def _split(n: int) -> int:
    """A factor n1 of n with 1 < n1 < n (the divisor closest to sqrt(n) from
    below), or 1 when n is prime."""
    best = 1
    d = 2
    while d * d <= n:
        if n % d == 0:
            best = d
        d += 1
    return best


def _dft_last(x: torch.Tensor, sign: int) -> torch.Tensor:
    """Unnormalised DFT along the last axis of a complex tensor."""
    n = x.shape[-1]
    n1 = _split(n)
    if n <= DIRECT or n1 == 1:
        return torch.matmul(x, _dft_matrix(n, sign).T)
    n2 = n // n1
    lead = x.shape[:-1]
    y = x.reshape(*lead, n1, n2).transpose(-1, -2)      # [j2][j1] = x(n2 j1 + j2)
    y = _dft_last(y, sign)                              # [j2][k1]
    y = y * _twiddle(n1, n2, sign)
    y = _dft_last(y.transpose(-1, -2), sign)            # [k1][k2]
    return y.transpose(-1, -2).reshape(*lead, n)        # index k1 + n1 k2


def _dft_mid(x: torch.Tensor, sign: int) -> torch.Tensor:
    """Unnormalised DFT along the middle axis of a contiguous [A][n][B]
    complex tensor: the same index map as ``_dft_last``, laid out so that
    the B values of one index move together (no strided gathers)."""
    a, n, b = x.shape
    n1 = _split(n)
    if n <= DIRECT or n1 == 1:
        return torch.matmul(_dft_matrix(n, sign), x)
    n2 = n // n1
    y = _dft_mid(x.reshape(a, n1, n2 * b), sign)        # [k1][j2] over j1 = x(n2 j1 + j2)
    y = y.reshape(a, n1, n2, b) * _twiddle(n1, n2, sign).T.reshape(1, n1, n2, 1)
    y = y.transpose(1, 2).reshape(a, n2, n1 * b)        # [j2][k1]
    y = _dft_mid(y, sign)                               # [k2][k1]: index k1 + n1 k2
    return y.reshape(a, n, b)


def dft(x: torch.Tensor, dim: int, inverse: bool = False) -> torch.Tensor:
    """DFT of a complex tensor along ``dim`` (F, or F^-1 with its 1/n)."""
    sign = 1 if inverse else -1
    dim = dim % x.dim()
    n = x.shape[dim]
    if dim == x.dim() - 1:
        y = _dft_last(x, sign)
    else:
        shape = x.shape
        a = math.prod(shape[:dim])
        b = math.prod(shape[dim + 1:])
        y = _dft_mid(x.contiguous().reshape(a, n, b), sign).reshape(shape)
    if inverse:
        y = y / n
    return y


def fftn(x: torch.Tensor) -> torch.Tensor:
    """3D F of a real or complex [n0][n1][n2] tensor (complex128 result)."""
    y = x.to(torch.complex128)
    for d in (2, 1, 0):
        y = dft(y, d)
    return y


def ifftn(x: torch.Tensor) -> torch.Tensor:
    """3D F^-1 (with 1/(n0 n1 n2)) of a complex tensor."""
    y = x.to(torch.complex128)
    for d in (0, 1, 2):
        y = dft(y, d, inverse=True)
    return y


def rfftn(x: torch.Tensor) -> torch.Tensor:
    """F of a real [n0][n1][n2] field, half spectrum [n0][n1][n2//2+1].

    The last axis is transformed first and cut to its non-negative modes;
    the other two axes are then transformed on the half spectrum."""
    n2 = x.shape[-1]
    y = dft(x.to(torch.complex128), 2)[..., : n2 // 2 + 1]
    return dft(dft(y, 1), 0)


def irfftn(h: torch.Tensor, s) -> torch.Tensor:
    """Real field [s0][s1][s2] whose F is the half spectrum ``h``.

    F^-1 along the first two axes, then along the last one on the line
    completed by X(-k) = conj X(k) (the relation of a real sequence), of
    which the real part is kept.  The imaginary parts of the m_z = 0 and
    m_z = s2/2 entries therefore drop out, as for any real inverse."""
    n2 = s[2]
    y = dft(dft(h.to(torch.complex128), 0, inverse=True), 1, inverse=True)
    half = n2 // 2 + 1
    if y.shape[-1] != half:
        raise ValueError(f"half spectrum has {y.shape[-1]} planes, expected {half}")
    tail = torch.conj(torch.flip(y[..., 1: n2 - half + 1], dims=(-1,)))
    full = torch.cat([y, tail], dim=-1)
    return dft(full, 2, inverse=True).real
