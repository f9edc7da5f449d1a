"""Plain FP64 CPU oracle for FFT-based 2LPT displacements in modified gravity.

TEST INFRASTRUCTURE ONLY.  This package is the slow, obviously correct
reference that the GPU path is checked against (Moretti, Mozzon, Monaco,
Munari & Baldi 2019, "Fast numerical method to generate halo catalogs in
modified gravity (part I): second-order Lagrangian Perturbation Theory").
Only ``tests/``, ``__graft_entry__.smoke()`` and the ``cpu_baseline`` leg of
``bench.py`` may import it.  It shares no code with the GPU library and
imports nothing from it; the only common input is the white noise drawn by
``seeded_inputs``.

Everything runs in float64 on the CPU (numpy for the growth ODE and the
background, torch CPU tensors for grid fields so that autograd can
differentiate the field pipeline).  The discrete Fourier transforms are the
oracle's own (``fft``: mixed-radix Cooley-Tukey in tensor operations, no FFT
library), pinned in ``tests/`` to the brute-force DFT.

Modules
    fft        -- the oracle's own 3D DFT (complex and real half spectrum)
    model      -- the parameter set (cosmology, gravity model, growth grid)
    cosmology  -- background, Hu-Sawicki m^2/M1/M2, mu(k,a), BBKS P(k), sigma8
    growth     -- the D1(k,a) and D2(k,a) ODEs (RK4 in ln a) and k tables
    fields     -- delta(k), psi1, phi_,ij, the source S, S(k), psi2
    spectrum   -- integer shell binning (mean, scatter, count, mean k)
    mgsource   -- the full MG source S1+S2+S3+S4, the ratio to GR, and the
                  choice of triangle configuration
    cic        -- cloud-in-cell painting of displaced particles and the loss
    adjoint    -- gradient of the CIC loss w.r.t. the white noise (autograd)

Readings of passages that are garbled, silent or inconsistent are listed in
the docstrings of the functions that take them.  Every function is pinned
by a test of tests/test_oracle_*.py; none is left "parity unpinned".
"""
from .model import Model, preset
from . import fft, cosmology, growth, fields, spectrum, mgsource, cic, adjoint

__all__ = ["Model", "preset", "fft", "cosmology", "growth", "fields", "spectrum",
           "mgsource", "cic", "adjoint"]
