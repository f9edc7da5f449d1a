"""Throughput of the 2LPT displacement path on one MI355X.

    python bench.py [--steps K] [--warmup W] [--gpus 1] [--no-cpu] [--no-fp64]

A step is one lpt2_displace call: the whole path from unit white noise to
psi1 and psi2 for one 512^3 realisation (L = 1024 Mpc/h, Hu-Sawicki n = 1),
cycling through |f_R0| in {1e-6, 1e-4}, z in {0, 1} and seeds 1-4 (16
combinations), FP32 fields with FP64 growth factors.  Inputs are resident in
HBM before the timed region; growth tables are built once per (model, a)
during warm-up (at least 16 steps: every combination once), outside the
timed region.  Prints one JSON line.

roofline: the launch site with the largest total time; its algorithmic
bytes per launch over its average duration from HIP events that the library
records around every launch on the launch stream during the timed steps
(that recording is extra host work inside the timed region; it does not
shorten the step).  step_achieved / step_frac: the same for the whole step
(all launch sites' algorithmic bytes over the event-timed step).
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

PEAK_HBM_GBS = 8000.0
N = 512
BOX = 1024.0
FR0S = (1e-6, 1e-4)
REDSHIFTS = (0.0, 1.0)
SEEDS = (1, 2, 3, 4)
CSRC = os.path.join(ROOT, "paper_1909_06282_amd", "csrc")
COPY_BYTES = 512 << 20


# the device code of the displacement passes (the counter readings describe
# those kernels; the host code, the growth and table kernels, the binner and
# the CIC kernels are left out)
KERNEL_SOURCES = ("cx.hpp", "fft_core.hpp", "fft_passes.hpp", "fft_kernels.hip", "kernels.hpp")

# the access shape of every launch site of the step: (kind, fields read,
# fields written, tile kind); kind 0 = contiguous lines (z passes), 1 = y
# columns, 2 = x columns; tile kind = the plan's tile list entry (0 single
# y FFT, 1 fused y, 2 fused x) that sets the site's columns per tile.  The
# pattern takes its tiles in the order the library's pass does: the fused y
# passes from per-XCD tickets at 128-byte rows, the fused x passes under 128
# bytes, the grid-stride order otherwise.
PATTERNS = {
    "z_r2c_noise": (0, 1, 1, None), "y_fwd_noise": (1, 1, 1, 0), "x_fused_psi1_phi": (2, 1, 5, 2),
    "y_inv_psi1_phi": (1, 5, 9, 1), "z_c2r_psi1": (0, 3, 3, None), "z_fused_source": (0, 6, 1, None),
    "y_fwd_source": (1, 1, 1, 0), "x_fused_psi2": (2, 1, 2, 2), "y_inv_psi2": (1, 2, 3, 1), "z_c2r_psi2": (0, 3, 3, None),
}


def source_hash() -> str:
    """Hash of the device code of the displacement passes."""
    h = hashlib.sha256()
    names = list(KERNEL_SOURCES) + sorted(f for f in os.listdir(CSRC) if f.startswith("fft_sizes_"))
    for f in names:
        with open(os.path.join(CSRC, f), "rb") as fh:
            h.update(f.encode() + fh.read())
    return h.hexdigest()[:16]


def pattern_rates(n: int, tiles, reps: int = 10):
    """Bandwidth of each launch site's access pattern with no arithmetic
    (libmembench.so: the same fields read and written, the same line or
    column-tile shape, `tiles` = the plan's [single y, fused y, fused x]
    widths): a reference for how far each site is from its traffic's rate."""
    import ctypes as C
    path = os.path.join(ROOT, "paper_1909_06282_amd", "libmembench.so")
    if not os.path.exists(path):
        return None
    lib = C.CDLL(path)
    lib.membench_pattern.argtypes = [C.c_int] * 6 + [C.POINTER(C.c_double)]
    lib.membench_pattern.restype = C.c_int
    out = {}
    for site, (kind, nin, nout, tk) in PATTERNS.items():
        ms = C.c_double(0.0)
        w = tiles[tk] if tk is not None else 16
        tickets = (tk == 1 and w * 8 >= 128) or (tk == 2 and w * 8 < 128)
        st = lib.membench_pattern(kind + (8 if tickets else 0), n, nin, nout, w, reps, C.byref(ms))
        if st != 0 or ms.value <= 0:
            out[site] = {"status": st}
            continue
        by = (nin + nout) * float(n) ** 3 * 4
        out[site] = {"kind": ("lines", "y columns", "x columns")[kind], "reads": nin, "writes": nout,
                     "columns_per_tile": w if tk is not None else None,
                     "order": "tickets" if tickets else "grid-stride",
                     "ms": round(ms.value, 4), "GBps": round(by / (ms.value / 1e3) / 1e9, 1)}
    return out


def attach_patterns(breakdown: dict, pat) -> None:
    """pattern_GBps / of_pattern beside each site's measured rate."""
    for site, c in (pat or {}).items():
        b = breakdown.get(site)
        if b and b.get("GBps") and c.get("GBps"):
            b["pattern_GBps"] = c["GBps"]
            b["of_pattern"] = round(b["GBps"] / c["GBps"], 3)


def traffic_for(kernel: str, launches_bytes: float):
    """HBM bytes per launch measured with rocprofv3 counters, if taken on this source."""
    path = os.path.join(ROOT, "profiles", "traffic.json")
    try:
        with open(path) as fh:
            rec = json.load(fh)
    except (OSError, ValueError):
        return None
    if rec.get("source_hash") != source_hash():
        return None
    k = rec.get("kernels", {}).get(kernel)
    return None if k is None else k.get("bytes_per_launch")


def traffic_from(fetch_dir: str, write_dir: str) -> None:
    """Write profiles/traffic.json and print its table from two rocprofv3 --pmc
    runs of this script (FETCH_SIZE, then WRITE_SIZE; default workload,
    --no-extra).  Each counter is scaled by its reading for the 512 MiB device
    copy of the same run; per launch site the median over the profiled steps."""
    import csv
    import glob
    import statistics

    def load(d, counter):
        f = glob.glob(os.path.join(d, "**", "*counter_collection.csv"), recursive=True)
        if not f:
            raise SystemExit(f"no counter_collection.csv under {d}")
        rows = {}
        with open(f[0]) as fh:
            for r in csv.DictReader(fh):
                if r["Counter_Name"] == counter:
                    rows.setdefault(int(r["Dispatch_Id"]), (r["Kernel_Name"], int(r["Grid_Size"]), float(r["Counter_Value"])))
        return [rows[k] for k in sorted(rows)]

    def per_site(disp):
        steps = []
        i = 0
        while i + len(PATTERNS) <= len(disp):
            if f"k_zr2c<float, {N}>" in disp[i][0]:
                steps.append(disp[i:i + len(PATTERNS)])
                i += len(PATTERNS)
            else:
                i += 1
        return {site: statistics.median(st[k][2] for st in steps) for k, site in enumerate(PATTERNS)}, len(steps)

    def scale(disp):
        copies = [d for d in disp if "copyBuffer" in d[0]]
        big = max(d[1] for d in copies)
        return COPY_BYTES / (statistics.median(d[2] for d in copies if d[1] == big) * 1024)

    fd, wd = load(fetch_dir, "FETCH_SIZE"), load(write_dir, "WRITE_SIZE")
    (fsite, nf), (wsite, nw) = per_site(fd), per_site(wd)
    fs, ws = scale(fd), scale(wd)
    kern = {}
    print("| launch site | fetched GB | written GB | total GB | algorithmic GB | total / algorithmic |")
    print("|---|---:|---:|---:|---:|---:|")
    for site, (kind, nin, nout, _) in PATTERNS.items():
        fb, wb = fsite[site] * 1024 * fs, wsite[site] * 1024 * ws
        alg = (nin + nout) * float(N) ** 3 * 4
        kern[site] = {"fetch_bytes": round(fb), "write_bytes": round(wb), "bytes_per_launch": round(fb + wb)}
        print(f"| {site} | {fb / 1e9:.3f} | {wb / 1e9:.3f} | {(fb + wb) / 1e9:.3f} | {alg / 1e9:.3f} | {(fb + wb) / alg:.3f} |")
    rec = {"source_hash": source_hash(), "workload": f"{N}^3 f(R) FP32 displacement (bench.py default workload)",
           "counter_runs": [fetch_dir, write_dir], "steps": [nf, nw],
           "scale": {"copy_bytes": COPY_BYTES, "fetch_scale": fs, "write_scale": ws,
                     "note": "bytes = counter KiB * 1024 * scale; scale = known copy bytes / counter reading "
                             "of the 512 MiB device copy in the same run"},
           "kernels": kern}
    with open(os.path.join(ROOT, "profiles", "traffic.json"), "w") as fh:
        json.dump(rec, fh, indent=1)
    print(f"source hash {rec['source_hash']}; steps {nf}/{nw}; scales {fs:.4f} {ws:.4f}")


def cpu_baseline(fr0: float, a: float, seed: int):
    """The FP64 oracle, as it is, on a bounded sample of the workload: one
    256^3 realisation at the headline's cell size (L = 512 Mpc/h, 2 Mpc/h
    cells) and gravity, on every host thread the process may use, then on one
    thread (the per-core figure).  Growth tables excluded, as on the GPU side."""
    import torch
    import oracle
    from oracle import fields, growth
    from seeded_inputs import white_noise
    n, box = N // 2, BOX / 2
    threads = int(os.environ.get("OMP_NUM_THREADS") or (os.cpu_count() or 1))
    threads = max(1, min(threads, os.cpu_count() or 1))
    m = oracle.Model(n=n, box=box, gravity="fr_hs", fr0_abs=fr0, factorisation="t1")
    tab = growth.tables(m, a)
    w = white_noise(n, seed)
    amp = oracle.cosmology.sigma8_amplitude(m)
    times = {}
    for nt in (threads, 1):
        torch.set_num_threads(nt)
        t0 = time.perf_counter()
        fields.displace(w, m, a, tab, amp)
        times[nt] = time.perf_counter() - t0
    torch.set_num_threads(threads)
    return {"value": n ** 3 / times[threads], "unit": "grid-cells/s", "cores": threads, "kind": "oracle",
            "sample": f"one {n}^3 realisation (L={box:.0f} Mpc/h, the headline's 2 Mpc/h cells), |f_R0|={fr0:g}, "
                      f"a={a}, seed {seed}; growth tables excluded; {times[threads]:.2f} s on {threads} threads",
            "single_thread": {"value": n ** 3 / times[1], "unit": "grid-cells/s", "seconds": round(times[1], 2)}}


def batched(steps: int, warmup: int):
    """The batched mix: 64 x 128^3 (L=256) + 32 x 64^3 (L=128), |f_R0| = 1e-5,
    z = 0, seeds 100-195, FP32; tiles from the tuner, the whole batch one
    captured graph per step."""
    import numpy as np
    import torch
    from paper_1909_06282_amd import LPT2Config, Plan
    from seeded_inputs import white_noise
    dev = torch.device("cuda:0")
    cfgs = [LPT2Config(n=128, box=256.0, gravity="fr_hs", fr0_abs=1e-5, factorisation="t1", precision="fp32"),
            LPT2Config(n=64, box=128.0, gravity="fr_hs", fr0_abs=1e-5, factorisation="t1", precision="fp32")]
    plan = Plan(cfgs, counts=[64, 32])
    sizes = [128] * 64 + [64] * 32
    noise = [torch.from_numpy(white_noise(n, s, np.float32)).to(dev) for n, s in zip(sizes, range(100, 196))]
    p1 = [torch.empty((3, n, n, n), dtype=torch.float32, device=dev) for n in sizes]
    p2 = [torch.empty_like(x) for x in p1]
    stream = torch.cuda.current_stream()
    t0 = time.perf_counter()
    tiles = plan.autotune(1.0, noise, p1, p2, stream=stream)
    tune_s = time.perf_counter() - t0
    cells = float(sum(n ** 3 for n in sizes))

    def timed(k):
        torch.cuda.synchronize()
        t = time.perf_counter()
        for _ in range(k):
            plan.displace(1.0, noise, p1, p2, stream=stream)
        torch.cuda.synchronize()
        return (time.perf_counter() - t) / k

    for _ in range(warmup):
        plan.displace(1.0, noise, p1, p2, stream=stream)
    eager = timed(max(4, steps // 2))
    plan.profile_reset()
    plan.profile_enable(True)
    plan.displace(1.0, noise, p1, p2, stream=stream)
    torch.cuda.synchronize()
    prof = {f"{name} [{by / 1e9:.3f} GB]": {"launches": launches, "avg_ms": round(ms / max(launches, 1), 4),
                                            "GBps": round(by / (ms / launches / 1e3) / 1e9, 1) if ms > 0 else None}
            for name, launches, ms, by in plan.profile()}
    plan.profile_enable(False)
    plan.set_graph(True)
    for _ in range(warmup):                    # first call captures the graph
        plan.displace(1.0, noise, p1, p2, stream=stream)
    graph = timed(steps)
    return {"workload": "64 x 128^3 (L=256) + 32 x 64^3 (L=128) realisations, Hu-Sawicki |f_R0|=1e-5, z=0, "
                        "seeds 100-195, FP32, one hipGraph launch per batch",
            "cells_per_batch": cells, "value": cells / graph, "unit": "grid-cells/s",
            "ms_per_batch": round(graph * 1e3, 4), "eager_ms_per_batch": round(eager * 1e3, 4),
            "steps": steps, "tiles": {"128": tiles[0], "64": tiles[1]}, "tune_s": round(tune_s, 2),
            "kernels_eager": prof}


def _timed(fn, reps):
    import torch
    fn()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(reps):
        fn()
    torch.cuda.synchronize()
    return (time.perf_counter() - t0) * 1e3 / reps


def adjoint_timing(reps: int):
    """The adjoint workload: 128^3 (L=256) f(R) |f_R0|=1e-5 FP32; loss = sum of
    squared residuals of the CIC density against the density of seed 7; one
    step = forward (displace, paint, loss) + backward (paint transpose,
    lpt2_backward) for the noise of seed 1."""
    import numpy as np
    import torch
    from paper_1909_06282_amd import Displace, LPT2Config, PaintCIC, Plan
    from seeded_inputs import white_noise
    plan = Plan(LPT2Config(n=128, box=256.0, gravity="fr_hs", fr0_abs=1e-5, factorisation="t1", precision="fp32"))
    with torch.no_grad():
        t1, t2 = plan.displace(1.0, torch.from_numpy(white_noise(128, 7, np.float32)).cuda())
        target = plan.paint_cic(t1, t2).clone()
    w = torch.from_numpy(white_noise(128, 1, np.float32)).cuda().requires_grad_(True)

    def step():
        w.grad = None
        p1, p2 = Displace.apply(w, plan, 1.0)
        loss = ((PaintCIC.apply(p1, p2, plan) - target) ** 2).sum()
        loss.backward()

    g1 = torch.randn((3, 128, 128, 128), device="cuda")
    g2 = torch.randn_like(g1)
    wd = w.detach()
    out = {"workload": "128^3 (L=256) f(R) |f_R0|=1e-5 FP32, CIC loss against seed 7, gradient for seed 1",
           "ms_loss_and_gradient": round(_timed(step, reps), 4),
           "ms_displace": round(_timed(lambda: plan.displace(1.0, wd), reps), 4),
           "ms_backward": round(_timed(lambda: plan.backward(1.0, wd, g1, g2), reps), 4)}
    plan.profile_reset()
    plan.profile_enable(True)
    for _ in range(reps):
        plan.backward(1.0, wd, g1, g2)
    torch.cuda.synchronize()
    prof = plan.profile()
    plan.profile_enable(False)
    tot_ms = sum(t for _, _, t, _ in prof) / reps
    tot_by = sum(by * l for _, l, _, by in prof) / reps
    out["backward_kernels"] = {f"{name} [{by / 1e9:.3f} GB]": {"avg_ms": round(t / l, 4),
                                                              "GBps": round(by / (t / l / 1e3) / 1e9, 1)}
                               for name, l, t, by in prof if t > 0}
    out["backward_algorithmic_GBps"] = round(tot_by / (tot_ms / 1e3) / 1e9, 1)
    out["backward_bytes_per_cell"] = round(tot_by / 128 ** 3, 1)
    return out


def epochs_timing(reps: int):
    """Four output times (z = 0, 0.5, 1, 2) of one 512^3 realisation (L=1024,
    |f_R0|=1e-6, FP32, seed 1) from one source, against four separate
    lpt2_displace calls."""
    import numpy as np
    import torch
    from paper_1909_06282_amd import LPT2Config, Plan
    from seeded_inputs import white_noise
    plan = Plan(LPT2Config(n=N, box=BOX, gravity="fr_hs", fr0_abs=1e-6, factorisation="t1", precision="fp32"))
    w = torch.from_numpy(white_noise(N, 1, np.float32)).cuda()
    a_list = [1.0, 1 / 1.5, 0.5, 1 / 3.0]
    o1 = [[torch.empty((3, N, N, N), dtype=torch.float32, device="cuda")] for _ in a_list]
    o2 = [[torch.empty((3, N, N, N), dtype=torch.float32, device="cuda")] for _ in a_list]
    t_ep = _timed(lambda: plan.displace_epochs(a_list, w, o1, o2), reps)

    def separate():
        for j, a in enumerate(a_list):
            plan.displace(a, w, o1[j][0], o2[j][0])
    t_sep = _timed(separate, reps)
    return {"workload": "512^3 (L=1024) |f_R0|=1e-6 FP32 seed 1 at z = 0, 0.5, 1, 2", "epochs": len(a_list),
            "ms_epochs_call": round(t_ep, 3), "ms_separate_calls": round(t_sep, 3),
            "value": len(a_list) * float(N) ** 3 / (t_ep / 1e3), "unit": "grid-cells/s"}


def grid_timing(n: int, box: float, reps: int, note: str, with_patterns: bool = False):
    """One realisation of the paper's own grid sizes: n^3 in `box` Mpc/h,
    |f_R0| = 1e-5, z = 0, FP32, with the per-kernel breakdown (and the
    memory-pattern reference of each site, where libmembench has the size)."""
    import numpy as np
    import torch
    from paper_1909_06282_amd import LPT2Config, Plan
    from seeded_inputs import white_noise
    plan = Plan(LPT2Config(n=n, box=box, gravity="fr_hs", fr0_abs=1e-5, factorisation="t1", precision="fp32"))
    w = torch.from_numpy(white_noise(n, 1, np.float32)).cuda()
    p1 = torch.empty((3, n, n, n), dtype=torch.float32, device="cuda")
    p2 = torch.empty_like(p1)
    plan.displace(1.0, w, p1, p2)
    plan.profile_reset()
    plan.profile_enable(True)
    ms = _timed(lambda: plan.displace(1.0, w, p1, p2), reps)
    prof = {name: {"avg_ms": round(t / max(l, 1), 4), "GBps": round(by / (t / l / 1e3) / 1e9, 1) if t > 0 else None}
            for name, l, t, by in plan.profile()}
    plan.profile_enable(False)
    tiles = plan.get_tiles(0)
    plan.close()
    del w, p1, p2
    torch.cuda.empty_cache()
    rec = {"workload": f"{n}^3 (L={box:g} Mpc/h) |f_R0|=1e-5 z=0 FP32 seed 1 ({note})", "ms_per_step": round(ms, 3),
           "value": float(n) ** 3 / (ms / 1e3), "unit": "grid-cells/s",
           "algorithmic_GBps": round(53 * 4 * float(n) ** 3 / (ms / 1e3) / 1e9, 1), "tiles": tiles, "kernels": prof}
    if with_patterns:
        pat = pattern_rates(n, tiles)
        if pat:
            attach_patterns(prof, pat)
            rec["patterns"] = pat
    return rec


def grid768_timing(reps: int, with_patterns: bool = True):
    """The paper's N-body grid: 768^3 in 750 Mpc/h (three times a power of
    two: a radix-12 first stage)."""
    return grid_timing(768, 750.0, reps, "radix-12 first stage", with_patterns)


def grid700_timing(reps: int):
    """The paper's 700 Mpc/h box at one particle per Mpc/h: 700^3 (x/y
    radices 5, 7, 4, 5; z 5, 7, 2, 5)."""
    return grid_timing(700, 700.0, reps, "radices 5 and 7")


def matter_power_timing(reps: int):
    """The matter power spectrum of the displaced particles at 512^3 (L=1024,
    |f_R0|=1e-6, z=0, FP32, seed 1): CIC paint of q + psi1 + psi2, forward 3D
    FFT, 256 shells with the CIC window divided out."""
    import numpy as np
    import torch
    from paper_1909_06282_amd import LPT2Config, Plan
    from seeded_inputs import white_noise
    plan = Plan(LPT2Config(n=N, box=BOX, gravity="fr_hs", fr0_abs=1e-6, factorisation="t1", precision="fp32"))
    w = torch.from_numpy(white_noise(N, 1, np.float32)).cuda()
    p1, p2 = plan.displace(1.0, w)
    delta = torch.empty((N, N, N), dtype=torch.float32, device="cuda")
    t_pk = _timed(lambda: plan.matter_power(p1, p2, 256, deconvolve=True), reps)
    t_int = _timed(lambda: plan.matter_power(p1, p2, 256, deconvolve=True, interlace=True), reps)
    t_paint = _timed(lambda: plan.paint_cic(p1, p2, delta), reps)
    return {"workload": "512^3 (L=1024) |f_R0|=1e-6 z=0 FP32 seed 1, 256 shells, CIC window divided out",
            "ms_matter_power": round(t_pk, 3), "ms_matter_power_interlaced": round(t_int, 3),
            "ms_cic_paint": round(t_paint, 3), "value": float(N) ** 3 / (t_pk / 1e3), "unit": "particles/s"}


def choice_timing(reps: int):
    """The factorisation choice at 256^3 (L=512) f(R) |f_R0|=1e-5 FP32, 128
    shells: the full MG source, its ratio to the GR source, the fit."""
    import numpy as np
    import torch
    from paper_1909_06282_amd import LPT2Config, Plan
    from seeded_inputs import white_noise
    plan = Plan(LPT2Config(n=256, box=512.0, gravity="fr_hs", fr0_abs=1e-5, factorisation="t1", precision="fp32"))
    w = torch.from_numpy(white_noise(256, 1, np.float32)).cuda()
    name = plan.choose_factorisation(1.0, w, nbins=128)[0]
    return {"workload": "256^3 (L=512) f(R) |f_R0|=1e-5 FP32, 128 shells, k <= 0.4 h/Mpc", "chosen": name,
            "ms_ratio_spectrum": round(_timed(lambda: plan.source_spectrum(1.0, w, 128, "ratio"), reps), 3),
            "ms_power_spectrum": round(_timed(lambda: plan.source_spectrum(1.0, w, 128, "power"), reps), 3),
            "ms_choice": round(_timed(lambda: plan.choose_factorisation(1.0, w, nbins=128), reps), 3)}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=32)
    ap.add_argument("--warmup", type=int, default=8)
    ap.add_argument("--no-cpu", action="store_true", help="skip the oracle baseline")
    ap.add_argument("--no-fp64", action="store_true", help="skip the FP64 companion measurement")
    ap.add_argument("--no-batch", action="store_true", help="skip the batched-mix measurement")
    ap.add_argument("--no-extra", action="store_true", help="skip the adjoint and factorisation-choice timings")
    ap.add_argument("--only-768", action="store_true",
                    help="time only the 768^3 grid (for profiling it) and print its record")
    ap.add_argument("--traffic-from", nargs=2, metavar=("FETCH_DIR", "WRITE_DIR"),
                    help="write profiles/traffic.json from two rocprofv3 --pmc runs (FETCH_SIZE, WRITE_SIZE) and exit")
    ap.add_argument("--only-700", action="store_true",
                    help="time only the 700^3 grid (for profiling it) and print its record")
    args = ap.parse_args()
    if args.traffic_from:
        traffic_from(*args.traffic_from)
        return
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) != 1:
        print("bench.py measures one GPU: the library has no multi-GPU path (run with --gpus 1)", file=sys.stderr)
        sys.exit(2)
    if args.only_768:
        print(json.dumps({"grid_768": grid768_timing(max(1, args.steps), with_patterns=False)}), flush=True)
        return
    if args.only_700:
        print(json.dumps({"grid_700": grid700_timing(max(1, args.steps))}), flush=True)
        return

    import numpy as np
    import torch
    from paper_1909_06282_amd import LPT2Config, Plan
    from seeded_inputs import white_noise

    dev = torch.device("cuda:0")
    combos = [(f, z, s) for f in FR0S for z in REDSHIFTS for s in SEEDS]

    def make_plans(prec):
        return {f: Plan(LPT2Config(n=N, box=BOX, gravity="fr_hs", fr0_abs=f, factorisation="t1",
                                   precision=prec)) for f in FR0S}

    # ---------------- FP32 headline ----------------
    plans = make_plans("fp32")
    noise = {s: torch.from_numpy(white_noise(N, s, np.float32)).to(dev) for s in SEEDS}
    psi1 = torch.empty((3, N, N, N), dtype=torch.float32, device=dev)
    psi2 = torch.empty_like(psi1)
    stream = torch.cuda.current_stream()

    def step(i):
        f, z, s = combos[i % len(combos)]
        plans[f].displace(1.0 / (1.0 + z), noise[s], psi1, psi2, stream=stream)

    warmup = max(args.warmup, len(combos))          # builds every (model, a) table once
    for i in range(warmup):
        step(i)
    torch.cuda.synchronize()
    for p in plans.values():
        p.profile_reset()
        p.profile_enable(True)
    ev0, ev1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    ev0.record(stream)
    for i in range(args.steps):
        step(i)
    ev1.record(stream)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    gpu_ms = ev0.elapsed_time(ev1)
    kernels = {}
    for p in plans.values():
        for name, launches, ms, by in p.profile():
            k = kernels.setdefault(name, [0, 0.0, by])
            k[0] += launches
            k[1] += ms
        p.profile_enable(False)
    tiles512 = plans[FR0S[0]].get_tiles(0)
    ms_per_step = wall * 1e3 / args.steps
    cells = float(N) ** 3
    value = cells * args.steps / wall
    step_bytes = sum(v[2] * v[0] for v in kernels.values()) / args.steps
    step_achieved = step_bytes / (gpu_ms / args.steps / 1e3) / 1e9
    dom = max(kernels.items(), key=lambda kv: kv[1][1])
    dname, (dl, dms, dbytes) = dom
    davg_s = dms / dl / 1e3
    achieved = dbytes / davg_s / 1e9
    breakdown = {k: {"launches": v[0], "avg_ms": round(v[1] / v[0], 4), "GB_per_launch": round(v[2] / 1e9, 4),
                     "GBps": round(v[2] / (v[1] / v[0] / 1e3) / 1e9, 1) if v[1] > 0 else None,
                     "share": round(v[1] / sum(x[1] for x in kernels.values()), 3)}
                 for k, v in sorted(kernels.items(), key=lambda kv: -kv[1][1])}

    # plain device copy of known size: context bandwidth, and the scale for the
    # FETCH_SIZE / WRITE_SIZE counters (512 MiB read + 512 MiB written)
    src = torch.empty(COPY_BYTES // 4, dtype=torch.float32, device=dev).fill_(1.0)
    dst = torch.empty_like(src)
    for _ in range(3):
        dst.copy_(src)
    torch.cuda.synchronize()
    c0 = time.perf_counter()
    for _ in range(10):
        dst.copy_(src)
    torch.cuda.synchronize()
    copy_gbs = 2 * COPY_BYTES * 10 / (time.perf_counter() - c0) / 1e9
    del src, dst

    # FP32 error against the FP64 GPU path (itself parity-tested against the oracle)
    extra = {}
    if not args.no_fp64:
        f, z, s = combos[0]
        plans[f].displace(1.0 / (1.0 + z), noise[s], psi1, psi2, stream=stream)
        torch.cuda.synchronize()
        ref32 = (psi1.clone(), psi2.clone())
        del plans, noise, psi1, psi2
        torch.cuda.empty_cache()
        p64 = make_plans("fp64")
        w64 = torch.from_numpy(white_noise(N, s)).to(dev)
        q1 = torch.empty((3, N, N, N), dtype=torch.float64, device=dev)
        q2 = torch.empty_like(q1)
        a = 1.0 / (1.0 + z)
        for _ in range(2):
            p64[f].displace(a, w64, q1, q2)
        torch.cuda.synchronize()
        k64 = max(4, args.steps // 4)
        t0 = time.perf_counter()
        for _ in range(k64):
            p64[f].displace(a, w64, q1, q2)
        torch.cuda.synchronize()
        w64t = time.perf_counter() - t0
        tot = (q1 + q2).abs().max().item()
        err = max((ref32[0].double() - q1).abs().max().item(), (ref32[1].double() - q2).abs().max().item())
        errt = ((ref32[0].double() + ref32[1].double()) - (q1 + q2)).abs().max().item()
        extra["fp64"] = {"value": cells * k64 / w64t, "ms_per_step": round(w64t * 1e3 / k64, 3), "steps": k64,
                         "config": f"|f_R0|={f:g}, z={z:g}, seed {s}"}
        extra["fp32_error_vs_fp64"] = {"max_abs_psi_component": err, "max_abs_total": errt,
                                       "normwise_total": errt / tot}
        del p64, q1, q2, w64
        torch.cuda.empty_cache()

    out = {
        "metric": "2LPT grid-cells/s at 512^3 f(R), FP32 vs FP64 at stated error; % HBM peak",
        "value": value,
        "unit": "grid-cells/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": warmup,
        "ms_per_step": round(ms_per_step, 4),
        "gpu_ms_per_step": round(gpu_ms / args.steps, 4),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": "512^3 grid, L=1024 Mpc/h, Hu-Sawicki n=1 |f_R0| in {1e-6,1e-4}, z in {0,1}, "
                               "seeds 1-4 (16 combinations cycled), T1 D2(k,a), FP32 fields, FP64 growth tables",
                   "grid": N, "box_mpc_h": BOX, "global_batch": 1, "parallelism": "single GPU"},
        "roofline": {"bound": "hbm", "kernel": dname, "achieved": round(achieved, 1), "peak": PEAK_HBM_GBS,
                     "unit": "GB/s", "frac": round(achieved / PEAK_HBM_GBS, 4),
                     "traffic": traffic_for(dname, dbytes), "bytes_per_launch": dbytes,
                     "avg_launch_ms": round(davg_s * 1e3, 4),
                     "step_achieved": round(step_achieved, 1), "step_frac": round(step_achieved / PEAK_HBM_GBS, 4)},
        "kernels": breakdown,
        "algorithmic_GBps_whole_step": round(step_achieved, 1),
        "torch_copy_GBps": round(copy_gbs, 1),
        "source_hash": source_hash(),
    }
    if not args.no_extra:
        pat = pattern_rates(N, tiles512)
        if pat:
            attach_patterns(breakdown, pat)
            c = pat.get(dname, {})
            if c.get("GBps"):
                out["roofline"]["pattern_GBps"] = c["GBps"]
                out["roofline"]["frac_of_pattern"] = round(achieved / c["GBps"], 4)
            out["patterns"] = pat
    out.update(extra)
    if not args.no_batch:
        out["batched"] = batched(max(8, args.steps // 2), 3)
        torch.cuda.empty_cache()
    if not args.no_extra:
        out["adjoint"] = adjoint_timing(8)
        out["factorisation_choice"] = choice_timing(3)
        out["matter_power"] = matter_power_timing(3)
        torch.cuda.empty_cache()
        out["epochs"] = epochs_timing(4)
        torch.cuda.empty_cache()
        out["grid_768"] = grid768_timing(5)
        torch.cuda.empty_cache()
        out["grid_700"] = grid700_timing(5)
        torch.cuda.empty_cache()
    out["numpy"] = np.__version__
    if not args.no_cpu:
        out["cpu_baseline"] = cpu_baseline(*combos[0][:1], 1.0, 1)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
