"""Pins of the oracle's FFT usage against a brute-force DFT and DFT identities.

The oracle calls torch.fft (pocketfft) for F and F^-1; these tests pin the
convention it relies on (unnormalised forward, 1/n^3 inverse, half spectrum
along the last axis) to the O(n^6) definition of the DFT.
"""
import numpy as np
import pytest
import torch

from seeded_inputs import white_noise


def brute_dft3(x: np.ndarray, sign: int) -> np.ndarray:
    n0, n1, n2 = x.shape
    out = np.zeros(x.shape, dtype=np.complex128)
    i0, i1, i2 = np.meshgrid(np.arange(n0), np.arange(n1), np.arange(n2), indexing="ij")
    for a in range(n0):
        for b in range(n1):
            for c in range(n2):
                ph = sign * 2j * np.pi * (a * i0 / n0 + b * i1 / n1 + c * i2 / n2)
                out[a, b, c] = np.sum(x * np.exp(ph))
    return out


@pytest.mark.parametrize("n", [8, 12])
def test_rfftn_matches_brute_force_dft(n):
    x = white_noise(n, 3)
    ref = brute_dft3(x, -1)[:, :, : n // 2 + 1]
    got = torch.fft.rfftn(torch.from_numpy(x)).numpy()
    assert np.max(np.abs(got - ref)) <= 1e-12 * np.max(np.abs(ref))


@pytest.mark.parametrize("n", [8])
def test_irfftn_matches_brute_force_inverse(n):
    x = white_noise(n, 4)
    full = brute_dft3(x, -1)
    back = brute_dft3(full, +1).real / n ** 3
    assert np.max(np.abs(back - x)) < 1e-12
    got = torch.fft.irfftn(torch.fft.rfftn(torch.from_numpy(x)), s=(n, n, n)).numpy()
    assert np.max(np.abs(got - x)) < 1e-12


def test_hermitian_symmetry_and_parseval():
    n = 16
    x = white_noise(n, 5)
    f = np.fft.fftn(x)
    neg = f[(-np.arange(n)) % n][:, (-np.arange(n)) % n][:, :, (-np.arange(n)) % n]
    assert np.max(np.abs(f - np.conj(neg))) < 1e-11
    assert abs(np.sum(x * x) - np.sum(np.abs(f) ** 2) / n ** 3) < 1e-10 * np.sum(x * x)
