"""Python binding of liblpt2 with the same entry points as the C ABI.

Argument marshalling only: every step runs in the HIP library.  Field
arguments are contiguous CUDA (HIP) torch tensors in the plan's precision;
the stream is torch's current stream unless one is given.
"""
from __future__ import annotations

import ctypes as C
from dataclasses import dataclass, fields as dc_fields
from typing import Sequence

import numpy as np
import torch

from . import _abi

_GRAVITY = {"gr": _abi.GRAV_GR, "fr_hs": _abi.GRAV_FR_HS, "mu_const": _abi.GRAV_MU_CONST}
_FACT = {"eds": _abi.D2_EDS, "t1": _abi.D2_T1, "triangle": _abi.D2_TRIANGLE,
         "winther": _abi.D2_WINTHER, "bouchet": _abi.D2_BOUCHET, "auto": _abi.D2_AUTO}
_PREC = {"fp64": _abi.FP64, "fp32": _abi.FP32}


@dataclass
class LPT2Config:
    """Mirror of lpt2_config with string enums."""
    n: int = 32
    box: float = 128.0
    omega_m: float = 0.3
    h: float = 0.7
    n_s: float = 0.96
    sigma8: float = 0.8
    gravity: str = "gr"
    fr0_abs: float = 1e-5
    hs_n: int = 1
    mu_const: float = 1.0
    factorisation: str = "eds"
    tri_ratio: float = 1.0
    tri_theta_deg: float = 90.0
    nk_growth: int = 256
    kmin: float = 1e-3
    kmax: float = 10.0
    a_init: float = 1e-3
    ode_steps: int = 4096
    precision: str = "fp64"

    def to_c(self) -> _abi.Config:
        c = _abi.Config()
        for f in dc_fields(self):
            v = getattr(self, f.name)
            if f.name == "gravity":
                v = _GRAVITY[v] if isinstance(v, str) else int(v)
            elif f.name == "factorisation":
                v = _FACT[v] if isinstance(v, str) else int(v)
            elif f.name == "precision":
                v = _PREC[v] if isinstance(v, str) else int(v)
            setattr(c, f.name, v)
        return c

    @property
    def dtype(self) -> torch.dtype:
        return torch.float32 if self.precision == "fp32" else torch.float64


def _stream(stream) -> C.c_void_p:
    if stream is None:
        return C.c_void_p(torch.cuda.current_stream().cuda_stream)
    if isinstance(stream, torch.cuda.Stream):
        return C.c_void_p(stream.cuda_stream)
    return C.c_void_p(int(stream))


def _ptrs(ts: Sequence[torch.Tensor]):
    arr = (C.c_void_p * len(ts))()
    for i, t in enumerate(ts):
        arr[i] = t.data_ptr()
    return arr


def factorisation_candidate(i: int):
    """(name, k1/k2 ratio, angle in degrees, winther) of candidate i."""
    L = _abi.load()
    nm, r, th, w = C.c_char_p(), C.c_double(), C.c_double(), C.c_int()
    _abi.check(L.lpt2_factorisation_candidate(int(i), C.byref(nm), C.byref(r), C.byref(th), C.byref(w)))
    return nm.value.decode(), r.value, th.value, bool(w.value)


class Plan:
    """Owns an lpt2 plan (workspace, twiddles, growth-table cache)."""

    def __init__(self, cfgs, counts: Sequence[int] | None = None):
        self._lib = _abi.load()
        if isinstance(cfgs, LPT2Config):
            cfgs = [cfgs]
        self.cfgs = list(cfgs)
        arr = (_abi.Config * len(self.cfgs))(*[c.to_c() for c in self.cfgs])
        cnt = None
        if counts is not None:
            cnt = (C.c_int * len(counts))(*counts)
        h = C.c_void_p()
        _abi.check(self._lib.lpt2_plan(arr, len(self.cfgs), cnt, C.byref(h)))
        self.handle = h
        self.dtype = self.cfgs[0].dtype
        self.sizes = []
        for r in range(self._lib.lpt2_realisations(h)):
            n = C.c_int()
            _abi.check(self._lib.lpt2_realisation_info(h, r, C.byref(n), None), h)
            self.sizes.append(n.value)

    def close(self):
        if getattr(self, "handle", None):
            self._lib.lpt2_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def _check_field(self, t: torch.Tensor, shape, what: str):
        if not isinstance(t, torch.Tensor) or not t.is_cuda:
            raise ValueError(f"{what} must be a device tensor")
        if t.dtype != self.dtype:
            raise ValueError(f"{what} must be {self.dtype}")
        if tuple(t.shape) != tuple(shape) or not t.is_contiguous():
            raise ValueError(f"{what} must be contiguous with shape {tuple(shape)}")

    def _lists(self, x):
        return [x] if isinstance(x, torch.Tensor) else list(x)

    def displace(self, a: float, noise, psi1=None, psi2=None, stream=None):
        """lpt2_displace; returns (psi1, psi2) (lists for multi-realisation plans)."""
        single = isinstance(noise, torch.Tensor)
        noise = self._lists(noise)
        if len(noise) != len(self.sizes):
            raise ValueError(f"plan holds {len(self.sizes)} realisations")
        if (psi1 is not None and len(self._lists(psi1)) != len(noise)) or \
                (psi2 is not None and len(self._lists(psi2)) != len(noise)):
            raise ValueError(f"plan holds {len(self.sizes)} realisations")
        if psi1 is None:
            psi1 = [torch.empty((3, n, n, n), dtype=self.dtype, device=w.device) for w, n in zip(noise, self.sizes)]
        if psi2 is None:
            psi2 = [torch.empty((3, n, n, n), dtype=self.dtype, device=w.device) for w, n in zip(noise, self.sizes)]
        psi1, psi2 = self._lists(psi1), self._lists(psi2)
        for w, p1, p2, n in zip(noise, psi1, psi2, self.sizes):
            self._check_field(w, (n, n, n), "noise")
            self._check_field(p1, (3, n, n, n), "psi1")
            self._check_field(p2, (3, n, n, n), "psi2")
        _abi.check(self._lib.lpt2_displace(self.handle, float(a), _ptrs(noise), _ptrs(psi1), _ptrs(psi2),
                                           _stream(stream)), self.handle)
        return (psi1[0], psi2[0]) if single else (psi1, psi2)

    def displace_noalloc(self, a: float, noise: torch.Tensor, psi1: torch.Tensor, psi2: torch.Tensor, stream=None):
        """lpt2_displace_noalloc: lpt2_displace of a one-realisation plan in the
        library's static scratch (the caller passes the outputs)."""
        n = self.sizes[0]
        self._check_field(noise, (n, n, n), "noise")
        self._check_field(psi1, (3, n, n, n), "psi1")
        self._check_field(psi2, (3, n, n, n), "psi2")
        _abi.check(self._lib.lpt2_displace_noalloc(self.handle, float(a), C.c_void_p(noise.data_ptr()),
                                                   C.c_void_p(psi1.data_ptr()), C.c_void_p(psi2.data_ptr()),
                                                   _stream(stream)), self.handle)
        return psi1, psi2

    def displace_epochs(self, a_list, noise, psi1=None, psi2=None, stream=None):
        """lpt2_displace_epochs: [(psi1, psi2) per a] (lists per realisation for multi-realisation plans)."""
        single = isinstance(noise, torch.Tensor)
        noise = self._lists(noise)
        a_list = [float(x) for x in a_list]
        R, E = len(self.sizes), len(a_list)
        if len(noise) != R:
            raise ValueError(f"plan holds {R} realisations")
        for w, n in zip(noise, self.sizes):
            self._check_field(w, (n, n, n), "noise")
        if psi1 is None:
            psi1 = [[torch.empty((3, n, n, n), dtype=self.dtype, device=w.device) for w, n in zip(noise, self.sizes)]
                    for _ in range(E)]
        if psi2 is None:
            psi2 = [[torch.empty((3, n, n, n), dtype=self.dtype, device=w.device) for w, n in zip(noise, self.sizes)]
                    for _ in range(E)]
        flat1 = [t for per in psi1 for t in self._lists(per)]
        flat2 = [t for per in psi2 for t in self._lists(per)]
        if len(flat1) != E * R or len(flat2) != E * R:
            raise ValueError("psi1/psi2 need one entry per (epoch, realisation)")
        for i, (p1, p2) in enumerate(zip(flat1, flat2)):
            n = self.sizes[i % R]
            self._check_field(p1, (3, n, n, n), "psi1")
            self._check_field(p2, (3, n, n, n), "psi2")
        arr = (C.c_double * E)(*a_list)
        _abi.check(self._lib.lpt2_displace_epochs(self.handle, E, arr, _ptrs(noise), _ptrs(flat1), _ptrs(flat2),
                                                  _stream(stream)), self.handle)
        out = []
        for j in range(E):
            o1, o2 = flat1[j * R:(j + 1) * R], flat2[j * R:(j + 1) * R]
            out.append((o1[0], o2[0]) if single else (o1, o2))
        return out

    def set_graph(self, enable: bool = True):
        """lpt2_set_graph: capture lpt2_displace into cached hipGraphs."""
        _abi.check(self._lib.lpt2_set_graph(self.handle, int(bool(enable))), self.handle)

    def tile_options(self, grid: int = 0):
        """[[widths of kind 0], [kind 1], [kind 2]]: the widths set_tiles accepts per pass kind."""
        w = (C.c_int * 9)()
        _abi.check(self._lib.lpt2_tile_options(self.handle, int(grid), w), self.handle)
        return [list(w[3 * k:3 * k + 3]) for k in range(3)]

    def get_tiles(self, grid: int = 0):
        w = (C.c_int * 3)()
        _abi.check(self._lib.lpt2_get_tiles(self.handle, int(grid), w), self.handle)
        return list(w)

    def set_tiles(self, grid: int, tiles):
        w = (C.c_int * 3)(*[int(x) for x in tiles])
        _abi.check(self._lib.lpt2_set_tiles(self.handle, int(grid), w), self.handle)

    def autotune(self, a: float, noise, psi1, psi2, cache_path: str | None = None, stream=None):
        """lpt2_autotune over the plan's realisations (buffers as for displace; overwritten)."""
        noise, psi1, psi2 = self._lists(noise), self._lists(psi1), self._lists(psi2)
        if not (len(noise) == len(psi1) == len(psi2) == len(self.sizes)):
            raise ValueError(f"plan holds {len(self.sizes)} realisations")
        for w, p1, p2, n in zip(noise, psi1, psi2, self.sizes):
            self._check_field(w, (n, n, n), "noise")
            self._check_field(p1, (3, n, n, n), "psi1")
            self._check_field(p2, (3, n, n, n), "psi2")
        path = None if cache_path is None else str(cache_path).encode()
        _abi.check(self._lib.lpt2_autotune(self.handle, float(a), _ptrs(noise), _ptrs(psi1), _ptrs(psi2), path,
                                           _stream(stream)), self.handle)
        return [self.get_tiles(g) for g in range(len(self.cfgs))]

    def backward(self, a: float, noise, g_psi1, g_psi2, g_noise=None, stream=None):
        """lpt2_backward: d/dw sum(g_psi1 psi1 + g_psi2 psi2)."""
        single = isinstance(noise, torch.Tensor)
        noise, g_psi1, g_psi2 = self._lists(noise), self._lists(g_psi1), self._lists(g_psi2)
        if g_noise is None:
            g_noise = [torch.empty_like(w) for w in noise]
        g_noise = self._lists(g_noise)
        R = len(self.sizes)
        if not (len(noise) == len(g_psi1) == len(g_psi2) == len(g_noise) == R):
            raise ValueError(f"plan holds {R} realisations: noise, g_psi1, g_psi2 and g_noise need one entry each")
        for w, a1, a2, gw, n in zip(noise, g_psi1, g_psi2, g_noise, self.sizes):
            self._check_field(w, (n, n, n), "noise")
            self._check_field(a1, (3, n, n, n), "g_psi1")
            self._check_field(a2, (3, n, n, n), "g_psi2")
            self._check_field(gw, (n, n, n), "g_noise")
        _abi.check(self._lib.lpt2_backward(self.handle, float(a), _ptrs(noise), _ptrs(g_psi1), _ptrs(g_psi2),
                                           _ptrs(g_noise), _stream(stream)), self.handle)
        return g_noise[0] if single else g_noise

    def source_spectrum(self, a: float, noise: torch.Tensor, nbins: int, quantity: str = "power", stream=None):
        """lpt2_source_spectrum -> dict of numpy arrays (k_mean, count, mean, std)."""
        n = self.sizes[0]
        self._check_field(noise, (n, n, n), "noise")
        q = _abi.SPEC_POWER if quantity == "power" else _abi.SPEC_RATIO
        out = [np.zeros(nbins) for _ in range(4)]
        ptr = [o.ctypes.data_as(C.POINTER(C.c_double)) for o in out]
        _abi.check(self._lib.lpt2_source_spectrum(self.handle, float(a), C.c_void_p(noise.data_ptr()), int(nbins), q,
                                                  *ptr, _stream(stream)), self.handle)
        return dict(zip(("k_mean", "count", "mean", "std"), out))

    def triangle_ratio(self, a: float, ratio: float, theta_deg: float, k, winther: bool = False):
        k = np.ascontiguousarray(k, dtype=np.float64)
        out = np.zeros_like(k)
        _abi.check(self._lib.lpt2_triangle_ratio(self.handle, float(a), float(ratio), float(theta_deg), int(winther),
                                                 k.ctypes.data_as(C.POINTER(C.c_double)), k.size,
                                                 out.ctypes.data_as(C.POINTER(C.c_double))), self.handle)
        return out

    def choose_factorisation(self, a: float, noise: torch.Tensor, nbins: int = 128, kcut: float = 0.4,
                             apply: bool = False, stream=None):
        """lpt2_choose_factorisation -> (candidate name, {name: cost})."""
        n = self.sizes[0]
        self._check_field(noise, (n, n, n), "noise")
        nc = self._lib.lpt2_factorisation_candidates()
        costs = (C.c_double * nc)()
        best = C.c_int()
        _abi.check(self._lib.lpt2_choose_factorisation(self.handle, float(a), C.c_void_p(noise.data_ptr()),
                                                       int(nbins), float(kcut), int(bool(apply)), C.byref(best),
                                                       costs, _stream(stream)), self.handle)
        names = [factorisation_candidate(i)[0] for i in range(nc)]
        return names[best.value], dict(zip(names, list(costs)))

    def auto_choice(self, grid: int, a: float):
        """Name of the candidate an AUTO configuration uses at a (None if not chosen yet)."""
        c = C.c_int()
        _abi.check(self._lib.lpt2_auto_choice(self.handle, int(grid), float(a), C.byref(c)), self.handle)
        return None if c.value < 0 else factorisation_candidate(c.value)[0]

    def displace_delta(self, a: float, delta: torch.Tensor, psi1=None, psi2=None, stream=None):
        """lpt2_displace_delta (test entry): psi1, psi2 from a real-space density contrast."""
        n = self.sizes[0]
        self._check_field(delta, (n, n, n), "delta")
        psi1 = torch.empty((3, n, n, n), dtype=self.dtype, device=delta.device) if psi1 is None else psi1
        psi2 = torch.empty((3, n, n, n), dtype=self.dtype, device=delta.device) if psi2 is None else psi2
        self._check_field(psi1, (3, n, n, n), "psi1")
        self._check_field(psi2, (3, n, n, n), "psi2")
        _abi.check(self._lib.lpt2_displace_delta(self.handle, float(a), C.c_void_p(delta.data_ptr()),
                                                 C.c_void_p(psi1.data_ptr()), C.c_void_p(psi2.data_ptr()),
                                                 _stream(stream)), self.handle)
        return psi1, psi2

    def matter_power(self, psi1: torch.Tensor, psi2: torch.Tensor, nbins: int, deconvolve: bool = False,
                     stream=None, interlace: bool = False):
        """lpt2_matter_power -> dict of numpy arrays (k_mean, count, mean, std);
        deconvolve divides out the CIC window, interlace averages with the
        painting half a cell over."""
        n = self.sizes[0]
        self._check_field(psi1, (3, n, n, n), "psi1")
        self._check_field(psi2, (3, n, n, n), "psi2")
        out = [np.zeros(nbins) for _ in range(4)]
        ptr = [o.ctypes.data_as(C.POINTER(C.c_double)) for o in out]
        _abi.check(self._lib.lpt2_matter_power(self.handle, C.c_void_p(psi1.data_ptr()), C.c_void_p(psi2.data_ptr()),
                                               int(nbins), int(bool(deconvolve)) | (2 if interlace else 0), *ptr,
                                               _stream(stream)), self.handle)
        return dict(zip(("k_mean", "count", "mean", "std"), out))

    def positions(self, psi1: torch.Tensor, psi2: torch.Tensor, r: int = 0, out=None, stream=None):
        """lpt2_positions: x = (q + psi1 + psi2) mod L for realisation r's particles."""
        n = self.sizes[r]
        self._check_field(psi1, (3, n, n, n), "psi1")
        self._check_field(psi2, (3, n, n, n), "psi2")
        out = torch.empty_like(psi1) if out is None else out
        self._check_field(out, (3, n, n, n), "pos")
        _abi.check(self._lib.lpt2_positions(self.handle, int(r), C.c_void_p(psi1.data_ptr()),
                                            C.c_void_p(psi2.data_ptr()), C.c_void_p(out.data_ptr()),
                                            _stream(stream)), self.handle)
        return out

    def check_finite(self, x: torch.Tensor, stream=None) -> int:
        """lpt2_check_finite: the number of non-finite values of a device
        tensor in the plan's precision (0 if every value is finite)."""
        if not isinstance(x, torch.Tensor) or not x.is_cuda or x.dtype != self.dtype or not x.is_contiguous():
            raise ValueError(f"expected a contiguous device tensor of {self.dtype}")
        cnt = C.c_longlong()
        st = self._lib.lpt2_check_finite(self.handle, C.c_void_p(x.data_ptr()), x.numel(), C.byref(cnt),
                                         _stream(stream))
        if st == _abi.EINVAL and cnt.value > 0:
            return int(cnt.value)
        _abi.check(st, self.handle)
        return int(cnt.value)

    def growth_table(self, a: float):
        nk = self.cfgs[0].nk_growth
        k, d1, d2 = np.zeros(nk), np.zeros(nk), np.zeros(nk)
        dp = C.POINTER(C.c_double)
        _abi.check(self._lib.lpt2_growth_table(self.handle, float(a), k.ctypes.data_as(dp), d1.ctypes.data_as(dp),
                                               d2.ctypes.data_as(dp)), self.handle)
        return k, d1, d2

    def fft3d(self, direction: int, x: torch.Tensor, stream=None) -> torch.Tensor:
        """Test entry lpt2_fft3d.  Forward returns complex [n][n][n/2]; inverse returns real n^3 F^-1."""
        n = self.sizes[0]
        if direction < 0:
            self._check_field(x, (n, n, n), "in")
            out = torch.empty((n, n, n // 2, 2), dtype=self.dtype, device=x.device)
        else:
            if x.is_complex():
                x = torch.view_as_real(x)
            self._check_field(x, (n, n, n // 2, 2), "in")
            out = torch.empty((n, n, n), dtype=self.dtype, device=x.device)
        _abi.check(self._lib.lpt2_fft3d(self.handle, int(direction), C.c_void_p(x.data_ptr()),
                                        C.c_void_p(out.data_ptr()), _stream(stream)), self.handle)
        return torch.view_as_complex(out) if direction < 0 else out

    def paint_cic(self, psi1, psi2, delta=None, stream=None) -> torch.Tensor:
        n = self.sizes[0]
        self._check_field(psi1, (3, n, n, n), "psi1")
        self._check_field(psi2, (3, n, n, n), "psi2")
        if delta is None:
            delta = torch.empty((n, n, n), dtype=self.dtype, device=psi1.device)
        self._check_field(delta, (n, n, n), "delta")
        _abi.check(self._lib.lpt2_paint_cic(self.handle, C.c_void_p(psi1.data_ptr()), C.c_void_p(psi2.data_ptr()),
                                            C.c_void_p(delta.data_ptr()), _stream(stream)), self.handle)
        return delta

    def paint_cic_backward(self, psi1, psi2, g_delta, g_psi=None, stream=None) -> torch.Tensor:
        n = self.sizes[0]
        self._check_field(psi1, (3, n, n, n), "psi1")
        self._check_field(psi2, (3, n, n, n), "psi2")
        self._check_field(g_delta, (n, n, n), "g_delta")
        if g_psi is None:
            g_psi = torch.empty((3, n, n, n), dtype=self.dtype, device=psi1.device)
        self._check_field(g_psi, (3, n, n, n), "g_psi")
        _abi.check(self._lib.lpt2_paint_cic_backward(self.handle, C.c_void_p(psi1.data_ptr()),
                                                     C.c_void_p(psi2.data_ptr()), C.c_void_p(g_delta.data_ptr()),
                                                     C.c_void_p(g_psi.data_ptr()), _stream(stream)), self.handle)
        return g_psi

    # ---- per-kernel timing ----
    def profile_enable(self, on: bool = True):
        _abi.check(self._lib.lpt2_profile_enable(self.handle, int(on)), self.handle)

    def profile_reset(self):
        _abi.check(self._lib.lpt2_profile_reset(self.handle), self.handle)

    def profile(self):
        """[(name, launches, total_ms, bytes_per_launch)] accumulated since the last reset."""
        out = []
        for i in range(self._lib.lpt2_profile_count(self.handle)):
            nm, ln, ms, by = C.c_char_p(), C.c_longlong(), C.c_double(), C.c_double()
            _abi.check(self._lib.lpt2_profile_get(self.handle, i, C.byref(nm), C.byref(ln), C.byref(ms),
                                                  C.byref(by)), self.handle)
            out.append((nm.value.decode(), ln.value, ms.value, by.value))
        return out

    def workspace_bytes(self) -> int:
        return int(self._lib.lpt2_workspace_bytes(self.handle))
