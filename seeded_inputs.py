"""Seeded synthetic inputs shared by the tests, the benchmark and the smoke check.

This module holds no arithmetic of the 2LPT method: it only draws the unit
Gaussian white noise that the method shapes into a density field, and the
index samples that tests use to pick cells.  Both the CPU oracle and the GPU
path receive the exact same arrays from here, so neither side draws random
numbers of its own.

Recipe: ``numpy.random.default_rng(seed).standard_normal((n, n, n))`` in
float64, C order (x slowest, z fastest); the float32 path receives the same
values rounded to float32.
"""
from __future__ import annotations

import numpy as np

__all__ = ["white_noise", "cell_sample", "realisation_seeds"]


def white_noise(n: int, seed: int, dtype=np.float64) -> np.ndarray:
    """Unit-variance white noise on an ``n^3`` grid, C order, from a PCG64 seed."""
    if n <= 0:
        raise ValueError("grid size must be positive")
    w = np.random.default_rng(seed).standard_normal((n, n, n))
    return np.ascontiguousarray(w.astype(dtype, copy=False))


def cell_sample(n: int, count: int, seed: int = 0) -> np.ndarray:
    """``count`` distinct flat cell indices of an ``n^3`` grid (no replacement)."""
    return np.random.default_rng(seed).choice(n ** 3, size=count, replace=False)


def realisation_seeds(first: int, count: int) -> list[int]:
    """Consecutive seeds for a batch of independent realisations."""
    return list(range(first, first + count))
