"""Batched form of the displacement path (through the C ABI).

Realisations of a plan are transformed a batch at a time (one launch per
pass for the whole batch), grids of different n on streams of their own, and
optionally as one captured hipGraph.  None of this changes the arithmetic
done for a realisation, so batched and graph results must be bitwise equal
to the single-realisation plan's; the single plans themselves are held to
the oracle (FP64 <= 1e-12 normwise) in test_gpu_parity.  Another tile width
is another instantiation of the same kernel template, where the compiler may
contract a different set of multiply-adds into FMAs, so across tile widths
results agree to rounding (a few ulp), not bitwise.
"""
import os

import numpy as np
import pytest
import torch

from oracle import fields, growth
from seeded_inputs import white_noise
from tests._util import gpu_config, normwise, oracle_model, to_dev

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module", autouse=True)
def _need_gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_1909_06282_amd import load_library
    load_library()


def _cfg(n, prec, **kw):
    base = dict(n=n, box=2.0 * n, gravity="fr_hs", fr0_abs=1e-5, factorisation="t1", nk_growth=64)
    base.update(kw)
    return gpu_config(precision=prec, **base)


ULP_TOL = {"fp32": 1e-6, "fp64": 1e-14}


def _close(got, ref, prec):
    return float((got.double() - ref.double()).abs().max() / ref.double().abs().max()) < ULP_TOL[prec]


def _single(cfg, a, w):
    from paper_1909_06282_amd import Plan
    return Plan(cfg).displace(a, w)


def _mixed(prec, counts=(5, 3), sizes=(16, 32), seed0=100):
    from paper_1909_06282_amd import Plan
    cfgs = [_cfg(n, prec) for n in sizes]
    plan = Plan(cfgs, counts=list(counts))
    dtype = cfgs[0].dtype
    noise, per = [], []
    s = seed0
    for cfg, cnt in zip(cfgs, counts):
        for _ in range(cnt):
            noise.append(to_dev(white_noise(cfg.n, s), dtype))
            per.append(cfg)
            s += 1
    return plan, cfgs, per, noise


@pytest.mark.parametrize("prec", ["fp64", "fp32"])
def test_batched_mixed_sizes_bitwise_equal_to_single(prec):
    print(f"batched 5x16^3 + 3x32^3 {prec}", flush=True)
    plan, cfgs, per, noise = _mixed(prec)
    p1, p2 = plan.displace(1.0, noise)
    torch.cuda.synchronize()
    for i, (cfg, w) in enumerate(zip(per, noise)):
        q1, q2 = _single(cfg, 1.0, w)
        torch.cuda.synchronize()
        assert torch.equal(p1[i], q1) and torch.equal(p2[i], q2), f"realisation {i}"
    if prec == "fp64":  # and one realisation of each grid against the oracle
        for i in (0, 5):
            m = oracle_model(per[i])
            r1, r2 = fields.displace(noise[i].cpu().numpy(), m, 1.0, growth.tables(m, 1.0))
            assert normwise(p1[i], r1) < 1e-12 and normwise(p2[i], r2) < 1e-12


def test_more_realisations_than_one_batch():
    # 70 realisations of 8^3: a batch of 64, then one of 6
    print("batched 70x8^3 fp64", flush=True)
    from paper_1909_06282_amd import Plan
    cfg = _cfg(8, "fp64")
    plan = Plan(cfg, counts=[70])
    noise = [to_dev(white_noise(8, 1000 + i), torch.float64) for i in range(70)]
    p1, p2 = plan.displace(0.5, noise)
    single = Plan(cfg)
    for i in range(70):
        q1, q2 = single.displace(0.5, noise[i])
        assert torch.equal(p1[i], q1) and torch.equal(p2[i], q2), f"realisation {i}"


def test_graph_replays_match_eager():
    # each replay is checked against the eager result, with eager work and
    # synchronisations between the replays
    print("graph replays 3x16^3 + 2x32^3 fp32", flush=True)
    plan, cfgs, per, noise = _mixed("fp32", counts=(3, 2))
    e1, e2 = plan.displace(1.0, noise)
    torch.cuda.synchronize()
    e1 = [x.clone() for x in e1]
    e2 = [x.clone() for x in e2]
    plan.set_graph(True)
    out1 = [torch.full_like(x, float("nan")) for x in e1]
    out2 = [torch.full_like(x, float("nan")) for x in e2]
    other = torch.randn(1 << 20, device="cuda")
    for rep in range(4):
        for x in out1 + out2:
            x.fill_(float("nan"))
        plan.displace(1.0, noise, out1, out2)
        other.mul_(1.0001).add_(0.5)          # eager work between replays
        torch.cuda.synchronize()
        for i in range(len(noise)):
            assert torch.equal(out1[i], e1[i]) and torch.equal(out2[i], e2[i]), f"replay {rep} realisation {i}"
    # other buffers -> a second graph; the first one still replays correctly
    alt1 = [torch.empty_like(x) for x in e1]
    alt2 = [torch.empty_like(x) for x in e2]
    plan.displace(1.0, noise, alt1, alt2)
    plan.displace(1.0, noise, out1, out2)
    torch.cuda.synchronize()
    for i in range(len(noise)):
        assert torch.equal(alt1[i], e1[i]) and torch.equal(alt2[i], e2[i])
        assert torch.equal(out1[i], e1[i]) and torch.equal(out2[i], e2[i])
    # another a -> another graph, equal to the eager path at that a
    plan.displace(0.5, noise, alt1, alt2)
    plan.set_graph(False)
    f1, f2 = plan.displace(0.5, noise)
    torch.cuda.synchronize()
    for i in range(len(noise)):
        assert torch.equal(alt1[i], f1[i]) and torch.equal(alt2[i], f2[i])


@pytest.mark.parametrize("prec", ["fp32", "fp64"])
def test_tile_widths_do_not_change_results(prec):
    print(f"tile widths {prec}", flush=True)
    plan, cfgs, per, noise = _mixed(prec, counts=(2, 2), sizes=(32, 64))
    ref1, ref2 = plan.displace(1.0, noise)
    torch.cuda.synchronize()
    ref1 = [x.clone() for x in ref1]
    ref2 = [x.clone() for x in ref2]
    for g in range(2):
        opts = plan.tile_options(g)
        for k in range(3):
            for w in sorted(set(opts[k])):
                t = plan.get_tiles(g)
                t[k] = w
                plan.set_tiles(g, t)
                q1, q2 = plan.displace(1.0, noise)
                torch.cuda.synchronize()
                for i in range(len(noise)):
                    assert _close(q1[i], ref1[i], prec) and _close(q2[i], ref2[i], prec), (g, k, w, i)
        plan.set_tiles(g, [0, 0, 0])


def test_set_tiles_rejects_widths_not_offered():
    from paper_1909_06282_amd import LPT2Error, Plan
    plan = Plan(_cfg(32, "fp32"))
    bad = max(max(o) for o in plan.tile_options(0)) * 2 + 1
    with pytest.raises(LPT2Error):
        plan.set_tiles(0, [bad, 0, 0])
    with pytest.raises(LPT2Error):
        plan.set_tiles(3, [0, 0, 0])


def test_autotune_picks_offered_tiles_and_caches_them(tmp_path):
    print("autotune 2x16^3 + 1x32^3", flush=True)
    from paper_1909_06282_amd import Plan
    plan, cfgs, per, noise = _mixed("fp32", counts=(2, 1))
    ref1, ref2 = plan.displace(1.0, noise)
    torch.cuda.synchronize()
    ref1 = [x.clone() for x in ref1]
    ref2 = [x.clone() for x in ref2]
    o1 = [torch.empty_like(x) for x in ref1]
    o2 = [torch.empty_like(x) for x in ref2]
    cache = tmp_path / "tiles.txt"
    tiles = plan.autotune(1.0, noise, o1, o2, cache_path=str(cache))
    lines = cache.read_text().splitlines()
    assert len(lines) == 2 and all(ln.startswith("lpt2-tiles ") for ln in lines)
    for g, t in enumerate(tiles):
        assert all(x in opts for x, opts in zip(t, plan.tile_options(g)))
    q1, q2 = plan.displace(1.0, noise)
    torch.cuda.synchronize()
    for i in range(len(noise)):
        assert _close(q1[i], ref1[i], "fp32") and _close(q2[i], ref2[i], "fp32")
    # a second plan of the same shape takes the cached entries without timing
    plan2 = Plan(cfgs, counts=[2, 1])
    assert plan2.autotune(1.0, noise, o1, o2, cache_path=str(cache)) == tiles
    assert cache.read_text().splitlines() == lines


@pytest.mark.parametrize("prec", ["fp64", "fp32"])
def test_epochs_equal_separate_displacements(prec):
    # the extra epochs reuse F[w] and F[S]; each epoch must equal a
    # separate lpt2_displace at its a (the same kernels and tables)
    print(f"epochs 2x16^3 + 1x32^3 {prec}", flush=True)
    plan, cfgs, per, noise = _mixed(prec, counts=(2, 1))
    a_list = [1.0, 0.5, 0.25, 2.0 / 3.0]
    outs = plan.displace_epochs(a_list, noise)
    torch.cuda.synchronize()
    for j, a in enumerate(a_list):
        q1, q2 = plan.displace(a, noise)
        torch.cuda.synchronize()
        for i in range(len(noise)):
            assert torch.equal(outs[j][0][i], q1[i]) and torch.equal(outs[j][1][i], q2[i]), (j, i)
    from paper_1909_06282_amd import LPT2Error
    with pytest.raises(LPT2Error):
        plan.displace_epochs([1.0] * 17, noise)
    # the largest number of epochs per call
    a16 = [1.0 / (1.0 + 0.2 * j) for j in range(16)]
    outs = plan.displace_epochs(a16, noise)
    torch.cuda.synchronize()
    for j in (0, 7, 15):
        q1, q2 = plan.displace(a16[j], noise)
        torch.cuda.synchronize()
        for i in range(len(noise)):
            assert torch.equal(outs[j][0][i], q1[i]) and torch.equal(outs[j][1][i], q2[i]), (j, i)


def test_batched_mixed_radix_and_power_of_two():
    # 3 x 96^3 (three times a power of two) beside 2 x 64^3, FP64
    print("batched 3x96^3 + 2x64^3 fp64", flush=True)
    plan, cfgs, per, noise = _mixed("fp64", counts=(3, 2), sizes=(96, 64))
    p1, p2 = plan.displace(1.0, noise)
    torch.cuda.synchronize()
    for i in (0, 2, 3):
        q1, q2 = _single(per[i], 1.0, noise[i])
        torch.cuda.synchronize()
        assert torch.equal(p1[i], q1) and torch.equal(p2[i], q2), f"realisation {i}"
