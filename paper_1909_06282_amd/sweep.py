"""Factorisation diagnostics across gravity strength and redshift.

For each (|f_R0|, z) of Hu-Sawicki n = 1 gravity, on one white-noise
realisation, this collects (Sec. 3, the triangle comparison, and Sec. 5,
the comparison with the LCDM fit of D2):

  * the shell-binned S_MG/S_GR of the full modified-gravity source (mean and
    1-sigma scatter per shell);
  * the analytic ratio R_T(k) of every candidate triangle at the shell mean
    wavenumbers, the count-weighted misfit of each over k <= kcut, and the
    chosen candidate;
  * on the growth-table nodes: D1(k,a), D2(k,a) of the T1 factorisation, and
    D2 of the LCDM fit (eq. lcdm-fit) and of GR.

Every number comes from the library's entry points (lpt2_source_spectrum,
lpt2_triangle_ratio, lpt2_choose_factorisation, lpt2_growth_table);
this module only loops and collects.  The caller supplies the white noise
(a device tensor); the command line draws unit Gaussian noise from a seed.

    python -m paper_1909_06282_amd.sweep --n 128 --box 256 \\
        --fr0 1e-4 1e-5 1e-6 --z 0 0.5 1 --out sweep.json
"""
from __future__ import annotations

import argparse
import json

import numpy as np
import torch

from .api import LPT2Config, Plan, factorisation_candidate


def candidates():
    """[(name, k1/k2, angle in degrees, winther)] in the library's order."""
    from . import _abi
    L = _abi.load()
    return [factorisation_candidate(i) for i in range(L.lpt2_factorisation_candidates())]


def sweep_point(noise: torch.Tensor, n: int, box: float, fr0: float, z: float, nbins: int, kcut: float = 0.4,
                precision: str = "fp64", **cosmo) -> dict:
    """The diagnostics of one (|f_R0|, z) for the given noise ([n][n][n] device tensor)."""
    a = 1.0 / (1.0 + z)
    base = dict(n=n, box=box, gravity="fr_hs", fr0_abs=fr0, precision=precision, **cosmo)
    plan = Plan(LPT2Config(factorisation="t1", **base))
    spec = plan.source_spectrum(a, noise, nbins, "ratio")
    sel = (spec["count"] > 0) & (spec["k_mean"] > 0) & (spec["k_mean"] <= kcut)
    k = spec["k_mean"][sel]
    curves = {name: plan.triangle_ratio(a, r, th, k, win).tolist() for name, r, th, win in candidates()}
    chosen, costs = plan.choose_factorisation(a, noise, nbins=nbins, kcut=kcut)
    kn, d1, d2 = plan.growth_table(a)
    fit = Plan(LPT2Config(factorisation="bouchet", **base)).growth_table(a)[2]
    gr = Plan(LPT2Config(n=n, box=box, gravity="gr", factorisation="t1", precision=precision, **cosmo)).growth_table(a)
    return {
        "fr0": fr0, "z": z, "a": a, "nbins": nbins, "kcut": kcut,
        "shells": {key: spec[key][sel].tolist() for key in ("k_mean", "count", "mean", "std")},
        "triangle_ratio": curves, "costs": costs, "chosen": chosen,
        "growth": {"k": kn.tolist(), "d1": d1.tolist(), "d2_t1": d2.tolist(), "d2_lcdm_fit": fit.tolist(),
                   "d1_gr": gr[1].tolist(), "d2_gr": gr[2].tolist()},
    }


def sweep(noise: torch.Tensor, box: float, fr0_list, z_list, nbins: int | None = None, kcut: float = 0.4,
          precision: str = "fp64", **cosmo) -> list:
    """sweep_point over every (|f_R0|, z), all on the same white noise
    (a contiguous [n][n][n] device tensor of the plan's precision)."""
    n = int(noise.shape[0])
    nb = nbins or n // 2
    return [sweep_point(noise, n, box, f, z, nb, kcut, precision, **cosmo) for f in fr0_list for z in z_list]


def main():
    ap = argparse.ArgumentParser(description=__doc__.split("\n\n")[0])
    ap.add_argument("--n", type=int, default=128)
    ap.add_argument("--box", type=float, default=256.0)
    ap.add_argument("--fr0", type=float, nargs="+", default=[1e-4, 1e-5, 1e-6])
    ap.add_argument("--z", type=float, nargs="+", default=[0.0, 0.5, 1.0])
    ap.add_argument("--seed", type=int, default=1)
    ap.add_argument("--nbins", type=int, default=None)
    ap.add_argument("--kcut", type=float, default=0.4)
    ap.add_argument("--precision", default="fp64", choices=["fp64", "fp32"])
    ap.add_argument("--out", default=None, help="write the records as JSON")
    args = ap.parse_args()
    dt = np.float32 if args.precision == "fp32" else np.float64
    w = np.random.default_rng(args.seed).standard_normal((args.n, args.n, args.n)).astype(dt)
    noise = torch.from_numpy(w).cuda()
    recs = sweep(noise, args.box, args.fr0, args.z, args.nbins, args.kcut, args.precision)
    for r in recs:
        best = sorted(r["costs"].items(), key=lambda kv: kv[1])[:3]
        g = r["growth"]
        i = int(np.argmin(np.abs(np.log(np.asarray(g["k"]) / 0.1))))
        print(f"|f_R0|={r['fr0']:g} z={r['z']:g}: chosen {r['chosen']:12s} "
              f"best {', '.join(f'{k} {v:.4g}' for k, v in best)}; at k={g['k'][i]:.3f}: D2_T1 "
              f"{g['d2_t1'][i]:.6g}, D2 of the LCDM fit {g['d2_lcdm_fit'][i]:.6g}", flush=True)
    if args.out:
        with open(args.out, "w") as fh:
            json.dump(recs, fh)


if __name__ == "__main__":
    main()
