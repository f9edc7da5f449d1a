"""The allocation-free entry point lpt2_displace_noalloc, called through the
C ABI, against lpt2_displace on the same inputs: two calls in a row on the
shared static scratch, the second with a smaller grid; tables built in the
scratch (no cached tables at a) and taken from the plan's cache; the size
limit refused on the host.  Bars: FP64 <= 1e-12, FP32 <= 1e-5 normwise
(the two use the same kernels and tables, so the results are also equal
bit for bit)."""
import ctypes as C

import numpy as np
import pytest
import torch

from seeded_inputs import white_noise
from tests._util import gpu_config, normwise, to_dev

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module", autouse=True)
def _need_gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")


def _noalloc(plan, a, w, p1, p2):
    from paper_1909_06282_amd import _abi
    L = _abi.load()
    st = L.lpt2_displace_noalloc(plan.handle, float(a), C.c_void_p(w.data_ptr()), C.c_void_p(p1.data_ptr()),
                                 C.c_void_p(p2.data_ptr()), C.c_void_p(torch.cuda.current_stream().cuda_stream))
    return st


def _case(prec, n, a, seed, tables_first):
    from paper_1909_06282_amd import Plan, _abi
    tol = 1e-12 if prec == "fp64" else 1e-5
    cfg = gpu_config(precision=prec, n=n, box=2.0 * n, gravity="fr_hs", fr0_abs=1e-5, factorisation="t1")
    plan = Plan(cfg)
    w = to_dev(white_noise(n, seed), cfg.dtype)
    q1 = torch.full((3, n, n, n), float("nan"), dtype=cfg.dtype, device="cuda")
    q2 = torch.full_like(q1, float("nan"))
    if tables_first:        # the plan caches its tables at a before the allocation-free call
        r1, r2 = plan.displace(a, w)
        assert _noalloc(plan, a, w, q1, q2) == _abi.OK, _abi.load().lpt2_last_error(plan.handle)
    else:                   # no cached tables: built in the scratch
        assert _noalloc(plan, a, w, q1, q2) == _abi.OK, _abi.load().lpt2_last_error(plan.handle)
        torch.cuda.synchronize()
        r1, r2 = plan.displace(a, w)
    torch.cuda.synchronize()
    e1, e2 = normwise(q1, r1), normwise(q2, r2)
    same = torch.equal(q1, r1) and torch.equal(q2, r2)
    print(f"  {prec} n={n} a={a} tables {'cached' if tables_first else 'in scratch'}: "
          f"psi1 {e1:.3e} psi2 {e2:.3e} bitwise {same}", flush=True)
    assert e1 <= tol and e2 <= tol
    assert same
    plan.close()


@pytest.mark.parametrize("prec", ["fp32", "fp64"])
def test_noalloc_equals_displace_two_calls_second_smaller(prec):
    big = 96 if prec == "fp32" else 64
    print(f"noalloc {prec}: n={big} then n=32", flush=True)
    _case(prec, big, 1.0, 3, tables_first=False)
    _case(prec, 32, 0.5, 4, tables_first=True)


def test_noalloc_refuses_beyond_its_scratch():
    from paper_1909_06282_amd import Plan, _abi
    print("noalloc size limit", flush=True)
    for prec, n in (("fp32", 128), ("fp64", 96)):
        cfg = gpu_config(precision=prec, n=n, box=2.0 * n, gravity="fr_hs", fr0_abs=1e-5, factorisation="t1")
        plan = Plan(cfg)
        w = torch.zeros((n, n, n), dtype=cfg.dtype, device="cuda")
        p1 = torch.zeros((3, n, n, n), dtype=cfg.dtype, device="cuda")
        st = _noalloc(plan, 1.0, w, p1, p1)
        msg = _abi.load().lpt2_last_error(plan.handle).decode()
        print(f"  {prec} n={n}: status {st}: {msg}", flush=True)
        assert st == _abi.EUNSUPPORTED and "scratch" in msg
        plan.close()
    from paper_1909_06282_amd import LPT2Config
    two = Plan([LPT2Config(n=16, box=32.0, precision="fp64")], counts=[2])
    w = torch.zeros((16, 16, 16), dtype=torch.float64, device="cuda")
    p1 = torch.zeros((3, 16, 16, 16), dtype=torch.float64, device="cuda")
    assert _noalloc(two, 1.0, w, p1, p1) == _abi.EUNSUPPORTED
    two.close()
