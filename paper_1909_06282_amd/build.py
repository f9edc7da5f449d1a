"""Build liblpt2.so (the HIP kernels for gfx950 and the C ABI) in-tree with hipcc,
and libmembench.so (memory-pattern ceilings for bench.py).

    python -m paper_1909_06282_amd.build        # or __graft_entry__.build()

Every source is compiled each time (a few tens of seconds, in parallel).
"""
from __future__ import annotations

import os
import shutil
import subprocess
import sys
from concurrent.futures import ThreadPoolExecutor

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(HERE, "csrc")
OUT = os.path.join(HERE, "liblpt2.so")
BUILD_DIR = os.path.join(HERE, "_build")
SOURCES = ["fft_kernels.hip", "aux_kernels.hip", "lpt2_api.cpp"] + sorted(
    f for f in os.listdir(CSRC) if f.startswith("fft_sizes_") and f.endswith(".hip"))
ARCH = "gfx950"

FLAGS = [
    "-O3", "-std=c++17", "-fPIC", f"--offload-arch={ARCH}",
    # packed FP32 instructions stay off (see the design notes)
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    "-Wall", "-Wno-unused-function", "-Wno-unused-command-line-argument",
    f"-I{os.path.join(os.path.dirname(HERE), 'include')}",
]


def hipcc() -> str:
    for cand in (shutil.which("hipcc"), "/opt/rocm/bin/hipcc"):
        if cand and os.path.exists(cand):
            return cand
    raise RuntimeError("hipcc not found")


def _compile(src: str) -> str:
    obj = os.path.join(BUILD_DIR, os.path.splitext(src)[0] + ".o")
    cmd = [hipcc(), "-x", "hip", *FLAGS, "-c", os.path.join(CSRC, src), "-o", obj]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError(f"compile of {src} failed:\n{' '.join(cmd)}\n{r.stdout}\n{r.stderr}")
    err = "\n".join(l for l in r.stderr.splitlines() if "packed-fp32-ops" not in l and l.strip())
    if err.strip():
        print(f"[{src}] {err}", file=sys.stderr)
    return obj


def build(verbose: bool = True) -> str:
    os.makedirs(BUILD_DIR, exist_ok=True)
    workers = max(1, min(len(SOURCES), int(os.environ.get("MAX_JOBS") or (os.cpu_count() or 1))))
    with ThreadPoolExecutor(max_workers=workers) as ex:
        objs = list(ex.map(_compile, SOURCES))
    tmp = OUT + ".tmp"
    cmd = [hipcc(), f"--offload-arch={ARCH}", "-shared", "-fPIC", *objs, "-o", tmp]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError(f"link failed:\n{' '.join(cmd)}\n{r.stdout}\n{r.stderr}")
    os.replace(tmp, OUT)
    # the memory-pattern ceilings that bench.py reports beside the passes
    mb = os.path.join(HERE, "libmembench.so")
    cmd = [hipcc(), "-x", "hip", *FLAGS, "-shared", os.path.join(CSRC, "membench.hip"), "-o", mb + ".tmp"]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError(f"membench build failed:\n{' '.join(cmd)}\n{r.stdout}\n{r.stderr}")
    os.replace(mb + ".tmp", mb)
    if verbose:
        print(f"built {OUT}")
    return OUT


if __name__ == "__main__":
    build()
