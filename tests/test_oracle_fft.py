"""Pins of the oracle's own DFT (oracle/fft.py) against the brute-force
definition of the DFT and against DFT identities.

The brute-force sum is the O(n^6) definition written out; it shares nothing
with the Cooley-Tukey splitting it checks.  Lengths cover every radix the
grids use (2, 3, 5, 7), a composite that splits twice (24 = 4 x 6), and a
prime (13, evaluated directly).  The library FFT (pocketfft, through numpy)
is used only as a second, independent cross-check at lengths too large for
the brute-force sum.
"""
import numpy as np
import pytest
import torch

from oracle import fft
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


def brute_dft1(x: np.ndarray, sign: int) -> np.ndarray:
    n = x.shape[-1]
    j = np.arange(n)
    w = np.exp(sign * 2j * np.pi * np.outer(j, j) / n)
    return x @ w.T


@pytest.mark.parametrize("n", [8, 10, 12, 14, 24])
def test_rfftn_matches_brute_force_dft(n):
    x = white_noise(n, 3)
    ref = brute_dft3(x, -1)[:, :, : n // 2 + 1]
    got = fft.rfftn(torch.from_numpy(x)).numpy()
    assert got.shape == ref.shape
    assert np.max(np.abs(got - ref)) <= 1e-13 * np.max(np.abs(ref))


@pytest.mark.parametrize("n", [8, 10, 14])
def test_complex_fftn_and_inverse_match_brute_force(n):
    rng = np.random.default_rng(11)
    x = rng.standard_normal((n, n, n)) + 1j * rng.standard_normal((n, n, n))
    ref = brute_dft3(x, -1)
    got = fft.fftn(torch.from_numpy(x)).numpy()
    assert np.max(np.abs(got - ref)) <= 1e-13 * np.max(np.abs(ref))
    back = fft.ifftn(torch.from_numpy(ref)).numpy()
    assert np.max(np.abs(back - brute_dft3(ref, +1) / n ** 3)) < 1e-13 * np.max(np.abs(x))
    assert np.max(np.abs(back - x)) < 1e-13 * np.max(np.abs(x))


@pytest.mark.parametrize("n", [8, 12, 14])
def test_irfftn_matches_brute_force_inverse(n):
    # a real field from its half spectrum: the brute-force inverse of the full
    # spectrum, real part (the imaginary part is zero to rounding)
    x = white_noise(n, 4)
    full = brute_dft3(x, -1)
    back = brute_dft3(full, +1) / n ** 3
    assert np.max(np.abs(back.imag)) < 1e-12
    got = fft.irfftn(torch.from_numpy(full[:, :, : n // 2 + 1]), s=(n, n, n)).numpy()
    assert np.max(np.abs(got - back.real)) < 1e-13
    assert np.max(np.abs(got - x)) < 1e-13


def test_irfftn_drops_imaginary_parts_of_self_conjugate_planes():
    # C2R semantics: an imaginary part on the m_z = 0 mode of a line whose
    # (x, y) modes are their own conjugates (here the DC column) cannot be
    # represented by a real field and must drop out
    n = 8
    h = np.zeros((n, n, n // 2 + 1), dtype=np.complex128)
    h[0, 0, 0] = 3.0 + 5.0j
    h[0, 0, n // 2] = 2.0 - 7.0j
    got = fft.irfftn(torch.from_numpy(h), s=(n, n, n)).numpy()
    z = np.arange(n)
    want = (3.0 + 2.0 * (-1.0) ** z) / n ** 3
    assert np.max(np.abs(got - want[None, None, :])) < 1e-15


@pytest.mark.parametrize("n", [2, 3, 5, 7, 13, 16, 17, 30, 42, 48, 60, 64, 96, 200, 350])
def test_one_dimensional_lengths_match_the_definition(n):
    rng = np.random.default_rng(n)
    x = rng.standard_normal((3, n)) + 1j * rng.standard_normal((3, n))
    ref = brute_dft1(x, -1)
    got = fft.dft(torch.from_numpy(x), 1).numpy()
    assert np.max(np.abs(got - ref)) <= 2e-14 * np.max(np.abs(ref)) * max(1.0, np.log2(n))
    inv = fft.dft(torch.from_numpy(ref), 1, inverse=True).numpy()
    assert np.max(np.abs(inv - x)) <= 2e-14 * np.max(np.abs(x)) * max(1.0, np.log2(n))


@pytest.mark.parametrize("n", [40, 56, 64, 96])
def test_cross_check_against_library_fft(n):
    x = white_noise(n, 6)
    got = fft.rfftn(torch.from_numpy(x)).numpy()
    ref = np.fft.rfftn(x)
    assert np.max(np.abs(got - ref)) <= 1e-13 * np.max(np.abs(ref))
    back = fft.irfftn(torch.from_numpy(ref), s=(n, n, n)).numpy()
    assert np.max(np.abs(back - x)) < 1e-13


def test_hermitian_symmetry_and_parseval():
    n = 16
    x = white_noise(n, 5)
    f = fft.fftn(torch.from_numpy(x)).numpy()
    neg = f[(-np.arange(n)) % n][:, (-np.arange(n)) % n][:, :, (-np.arange(n)) % n]
    assert np.max(np.abs(f - np.conj(neg))) < 1e-11
    assert abs(np.sum(x * x) - np.sum(np.abs(f) ** 2) / n ** 3) < 1e-10 * np.sum(x * x)


def test_autograd_through_the_transform_is_the_adjoint():
    # <F x, y> = <x, F^H y>: the gradient of Re<F x, y> w.r.t. real x is
    # Re(F^H y), and F^H = n^3 F^-1
    n = 10
    x = torch.from_numpy(white_noise(n, 8)).requires_grad_(True)
    rng = np.random.default_rng(9)
    y = torch.from_numpy(rng.standard_normal((n, n, n)) + 1j * rng.standard_normal((n, n, n)))
    obj = (fft.fftn(x) * y.conj()).real.sum()
    obj.backward()
    want = (fft.ifftn(y) * n ** 3).real
    assert float((x.grad - want).abs().max()) < 1e-12 * float(want.abs().max())
