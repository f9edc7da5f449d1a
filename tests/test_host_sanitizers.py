"""The host code of the C ABI under AddressSanitizer and
UndefinedBehaviorSanitizer (host side only: the device code is built as
usual).  tests/sanitize_driver.cpp walks every validation and error path
that runs without a device -- refused configurations, a plan whose first
allocation fails, NULL plans on the entry points, status strings, the
candidate table -- and the sanitizers turn any memory error or undefined
behaviour on those paths into a failure.  Uses the device-code objects of
the last in-tree build (paper_1909_06282_amd/_build)."""
import glob
import os
import shutil
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
CSRC = os.path.join(ROOT, "paper_1909_06282_amd", "csrc")
BUILD = os.path.join(ROOT, "paper_1909_06282_amd", "_build")
SAN = ["-Xarch_host", "-fsanitize=address", "-Xarch_host", "-fsanitize=undefined",
       "-Xarch_host", "-fno-sanitize-recover=undefined"]


def _hipcc():
    for cand in (shutil.which("hipcc"), "/opt/rocm/bin/hipcc"):
        if cand and os.path.exists(cand):
            return cand
    pytest.skip("hipcc not found")


def test_host_code_under_address_and_undefined_behaviour_sanitizers(tmp_path):
    hipcc = _hipcc()
    objs = [os.path.join(BUILD, f) for f in ("aux_kernels.o", "fft_kernels.o")]
    objs += sorted(glob.glob(os.path.join(BUILD, "fft_sizes_*.o")))
    if not all(os.path.exists(o) for o in objs) or len(objs) < 3:
        pytest.skip("device-code objects not built (run the in-tree build first)")
    inc = f"-I{os.path.join(ROOT, 'include')}"
    api = str(tmp_path / "api_san.o")
    drv = str(tmp_path / "drv.o")
    exe = str(tmp_path / "sanitize_driver")
    steps = [
        [hipcc, "-x", "hip", "--offload-arch=gfx950", "-O1", "-g", "-std=c++17", "-fPIC",
         "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops", *SAN, inc,
         "-c", os.path.join(CSRC, "lpt2_api.cpp"), "-o", api],
        [hipcc, "-O1", "-g", "-std=c++17", *SAN, inc, "-c", os.path.join(ROOT, "tests", "sanitize_driver.cpp"),
         "-o", drv],
        [hipcc, "--offload-arch=gfx950", *SAN[:4], drv, api, *objs, "-o", exe],
    ]
    for cmd in steps:
        r = subprocess.run(cmd, capture_output=True, text=True)
        assert r.returncode == 0, f"{' '.join(cmd)}\n{r.stdout}\n{r.stderr}"
    env = dict(os.environ, ASAN_OPTIONS="detect_leaks=0", UBSAN_OPTIONS="print_stacktrace=1")
    r = subprocess.run([exe], capture_output=True, text=True, env=env, timeout=300)
    print(r.stdout[-2000:])
    assert r.returncode == 0, r.stdout[-4000:] + r.stderr[-4000:]
    assert "SANITIZE DRIVER OK" in r.stdout
    assert "runtime error" not in r.stderr and "AddressSanitizer" not in r.stderr
