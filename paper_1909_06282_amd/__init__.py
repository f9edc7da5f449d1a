"""MI355X (gfx950) 2LPT displacements in modified gravity.

The FFT-based second-order Lagrangian pipeline of Moretti et al. (2019):
white noise shaped by sqrt(P(k)), first-order displacement with the
scale-dependent D1(k,a), the six potential derivatives and the second-order
source S, its FFT and shell spectrum, and the second-order displacement with
a k-dependent D2(k,a).  All steps run in hand-written HIP kernels behind the
C ABI of include/lpt2.h (liblpt2.so, built in-tree by ``build.py``); this
package only marshals arguments.
"""
from .api import LPT2Config, Plan, factorisation_candidate
from ._abi import LPT2Error, load as load_library
from .autograd import Displace, PaintCIC

__all__ = ["LPT2Config", "Plan", "LPT2Error", "load_library", "Displace", "PaintCIC", "factorisation_candidate"]
