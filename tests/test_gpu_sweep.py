"""The factorisation sweep: its records equal the oracle's on the same noise."""
import numpy as np
import pytest
import torch

from oracle import growth, mgsource
from seeded_inputs import white_noise
from tests._util import gpu_config, oracle_model

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module", autouse=True)
def _need_gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")


def test_sweep_point_matches_oracle():
    print("sweep 32^3, |f_R0| in {1e-4, 1e-5}, z in {0, 1}", flush=True)
    from paper_1909_06282_amd import sweep
    n, box, nb = 32, 128.0, 16
    w = white_noise(n, 3)
    recs = sweep.sweep(torch.from_numpy(w).cuda(), box, [1e-4, 1e-5], [0.0, 1.0], nbins=nb, nk_growth=64)
    assert len(recs) == 4
    for r in recs:
        cfg = gpu_config(n=n, box=box, gravity="fr_hs", fr0_abs=r["fr0"], factorisation="t1", nk_growth=64)
        m = oracle_model(cfg)
        tab = growth.tables(m, r["a"])
        km, cnt, mean, std = mgsource.source_ratio(w, m, r["a"], nb, tab)
        best, costs = mgsource.choose_triangle(km, cnt, mean, m, r["a"], 0.4, tab)
        sel = (cnt > 0) & (km > 0) & (km <= 0.4)
        assert np.allclose(r["shells"]["mean"], mean[sel], rtol=0, atol=1e-10)
        assert r["chosen"] == best
        for name, v in costs.items():
            assert abs(r["costs"][name] - v) <= 1e-8 * max(1.0, abs(v))
        # T1 curve against the oracle's analytic ratio at the same wavenumbers
        rt = mgsource.triangle_ratio(np.asarray(r["shells"]["k_mean"]), m, r["a"], 1.0, 90.0, tab=tab)
        assert np.allclose(r["triangle_ratio"]["T1"], rt, rtol=1e-11, atol=0)
        # D2 over the LCDM fit on the nodes
        fit = growth.tables(m.with_(factorisation="bouchet"), r["a"])[2]
        assert np.allclose(r["growth"]["d2_t1"], tab[2], rtol=1e-11, atol=0)
        assert np.allclose(r["growth"]["d2_lcdm_fit"], fit, rtol=1e-11, atol=0)
        print(f"  |f_R0|={r['fr0']:g} z={r['z']:g}: chosen {r['chosen']} (oracle {best})", flush=True)
