"""GPU parity of the HIP path (through the C ABI) against the FP64 oracle.

Bars: FP64 path <= 1e-12 normwise (max |gpu - oracle| / max |oracle|),
FP32 path <= 1e-5 normwise, integer bin counts exact, binner bitwise
reproducible.  Sizes 8^3..128^3 cover several tiles and the ragged tails of
the small grids (partial blocks of lines and columns).
"""
import math

import numpy as np
import pytest
import torch

import oracle
from oracle import adjoint, cic, fields, growth, mgsource, spectrum
from seeded_inputs import white_noise
from tests._util import gpu_config, normwise, oracle_model, to_dev

pytestmark = pytest.mark.gpu

F64_TOL = 1e-12
F32_TOL = 1e-5


@pytest.fixture(scope="module", autouse=True)
def _need_gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_1909_06282_amd import load_library
    load_library()


def _plan(**kw):
    from paper_1909_06282_amd import Plan
    cfg = gpu_config(**kw)
    return Plan(cfg), cfg


_TAB_CACHE = {}


def _tables(model, a):
    key = (model, a)
    if key not in _TAB_CACHE:
        _TAB_CACHE[key] = growth.tables(model, a)
    return _TAB_CACHE[key]


# ---------------------------------------------------------------- FFT
@pytest.mark.parametrize("prec", ["fp64", "fp32"])
@pytest.mark.parametrize("n", [8, 16, 32, 64, 128, 24, 48, 96, 40, 56, 200])
def test_fft3d_forward_matches_dft(n, prec):
    print(f"fft3d forward n={n} {prec}", flush=True)
    plan, cfg = _plan(precision=prec, n=n, box=2.0 * n)
    x = white_noise(n, 5)
    got = plan.fft3d(-1, to_dev(x, cfg.dtype)).cpu().to(torch.complex128)
    ref = oracle.fft.rfftn(torch.from_numpy(x))[:, :, : n // 2]
    err = float((got - ref).abs().max() / ref.abs().max())
    assert err < (1e-14 if prec == "fp64" else 1e-6), err


@pytest.mark.parametrize("prec", ["fp64", "fp32"])
@pytest.mark.parametrize("n", [8, 16, 32, 64, 128, 24, 48, 96, 40, 56, 200])
def test_fft3d_inverse_matches_dft(n, prec):
    print(f"fft3d inverse n={n} {prec}", flush=True)
    plan, cfg = _plan(precision=prec, n=n, box=2.0 * n)
    x = white_noise(n, 6)
    half = oracle.fft.rfftn(torch.from_numpy(x))
    half[:, :, n // 2] = 0
    ref = oracle.fft.irfftn(half, s=(n, n, n)) * n ** 3
    inp = torch.view_as_real(half[:, :, : n // 2].contiguous()).to(cfg.dtype).cuda().contiguous()
    got = plan.fft3d(+1, inp).cpu()
    assert normwise(got, ref) < (1e-14 if prec == "fp64" else 1e-6)


# ---------------------------------------------------------------- growth
@pytest.mark.parametrize("kw", [
    dict(gravity="gr", factorisation="eds"),
    dict(gravity="gr", factorisation="t1"),
    dict(gravity="fr_hs", fr0_abs=1e-5, factorisation="t1"),
    dict(gravity="fr_hs", fr0_abs=1e-4, factorisation="winther"),
    dict(gravity="fr_hs", fr0_abs=1e-6, factorisation="triangle", tri_ratio=2.0, tri_theta_deg=70.0),
    dict(gravity="fr_hs", fr0_abs=1e-5, factorisation="bouchet"),
    dict(gravity="mu_const", mu_const=4.0 / 3.0, omega_m=1.0, factorisation="t1"),
])
@pytest.mark.parametrize("a", [1.0, 0.5])
def test_growth_table_matches_oracle(kw, a):
    print(f"growth {kw} a={a}", flush=True)
    plan, cfg = _plan(n=8, box=16.0, nk_growth=64, **kw)
    k, d1, d2 = plan.growth_table(a)
    kn, o1, o2 = _tables(oracle_model(cfg), a)
    assert np.max(np.abs(k / kn - 1)) < 1e-14
    assert np.max(np.abs(d1 / o1 - 1)) < 1e-12
    assert np.max(np.abs(d2 / o2 - 1)) < 1e-12


@pytest.mark.parametrize("nk", [2, 62, 63, 126, 256, 1023])
def test_growth_table_node_counts(nk):
    # the growth kernel runs 63 nodes per one-wave block (its last lane the
    # normalisation run): the smallest and largest node counts, one lane
    # short of a block, exact multiples of a block, the default
    print(f"growth nk={nk}", flush=True)
    plan, cfg = _plan(n=8, box=16.0, nk_growth=nk, gravity="fr_hs", fr0_abs=1e-5, factorisation="t1")
    k, d1, d2 = plan.growth_table(0.8)
    kn, o1, o2 = _tables(oracle_model(cfg), 0.8)
    assert len(k) == nk
    assert np.max(np.abs(k / kn - 1)) < 1e-14
    assert np.max(np.abs(d1 / o1 - 1)) < 1e-12
    assert np.max(np.abs(d2 / o2 - 1)) < 1e-12


# ---------------------------------------------------------------- displacements
def _check_displace(prec, a, tol, seed=1, **kw):
    plan, cfg = _plan(precision=prec, **kw)
    model = oracle_model(cfg)
    w = white_noise(cfg.n, seed)
    p1, p2 = plan.displace(a, to_dev(w, cfg.dtype))
    torch.cuda.synchronize()
    r1, r2 = fields.displace(w, model, a, _tables(model, a))
    e1, e2 = normwise(p1, r1), normwise(p2, r2)
    tot = normwise(p1.double() + p2.double(), r1 + r2)
    print(f"  psi1 {e1:.3e} psi2 {e2:.3e} total {tot:.3e}", flush=True)
    assert e1 < tol and e2 < tol and tot < tol
    return plan, cfg, p1, p2


def test_displace_c1_gr_fp64():
    print("displace C1 GR fp64", flush=True)
    _check_displace("fp64", 1.0, F64_TOL, n=32, box=128.0, gravity="gr", factorisation="eds")


@pytest.mark.parametrize("n", [8, 16, 32, 64, 24, 48, 96, 192])
@pytest.mark.parametrize("a", [1.0, 0.5])
def test_displace_fr_t1_fp64(n, a):
    print(f"displace f(R) T1 fp64 n={n} a={a}", flush=True)
    _check_displace("fp64", a, F64_TOL, n=n, box=2.0 * n, gravity="fr_hs", fr0_abs=1e-5,
                    factorisation="t1", nk_growth=64)


@pytest.mark.parametrize("n", [40, 56])
@pytest.mark.parametrize("a", [1.0, 0.5])
def test_displace_radix57_fp64(n, a):
    # grids with a factor 5 (40: x/y radices 8, 5; z 5, 4) and 7 (56: 8, 7;
    # z 7, 4), 1 Mpc/h cells as in the paper's source-ratio boxes
    print(f"displace f(R) T1 fp64 n={n} a={a}", flush=True)
    _check_displace("fp64", a, F64_TOL, n=n, box=float(n), gravity="fr_hs", fr0_abs=1e-4,
                    factorisation="t1", nk_growth=64)


@pytest.mark.parametrize("n", [8, 32, 128, 96, 40, 56])
def test_displace_fr_t1_fp32(n):
    print(f"displace f(R) T1 fp32 n={n}", flush=True)
    _check_displace("fp32", 1.0, F32_TOL, n=n, box=2.0 * n, gravity="fr_hs", fr0_abs=1e-5,
                    factorisation="t1", nk_growth=64)


@pytest.mark.parametrize("prec,tol", [("fp64", F64_TOL), ("fp32", F32_TOL)])
def test_displace_epochs_match_oracle(prec, tol):
    # lpt2_displace_epochs: the full chain at the first a, the first-order x
    # pass and the psi2 passes from the kept F[w], F[S] at the others; every
    # output time against the oracle (the factorisation of the unevolved
    # potential, Sec. 2.4)
    print(f"epochs vs oracle {prec} n=32", flush=True)
    plan, cfg = _plan(precision=prec, n=32, box=64.0, gravity="fr_hs", fr0_abs=1e-5, factorisation="t1",
                      nk_growth=64)
    m = oracle_model(cfg)
    w = white_noise(32, 5)
    a_list = [1.0, 2.0 / 3.0, 0.5, 0.25]
    outs = plan.displace_epochs(a_list, to_dev(w, cfg.dtype))
    torch.cuda.synchronize()
    for (p1, p2), a in zip(outs, a_list):
        r1, r2 = fields.displace(w, m, a, _tables(m, a))
        e1, e2 = normwise(p1, r1), normwise(p2, r2)
        tot = normwise(p1.double() + p2.double(), r1 + r2)
        print(f"  a={a:.4f}: psi1 {e1:.3e} psi2 {e2:.3e} total {tot:.3e}", flush=True)
        assert e1 < tol and e2 < tol and tot < tol
    plan.close()


def test_displace_batched_plan_matches_single():
    print("displace two-grid plan", flush=True)
    from paper_1909_06282_amd import Plan
    c1 = gpu_config(n=32, box=64.0, gravity="fr_hs", fr0_abs=1e-5, factorisation="t1", nk_growth=64)
    c2 = gpu_config(n=16, box=32.0, gravity="fr_hs", fr0_abs=1e-5, factorisation="t1", nk_growth=64)
    plan = Plan([c1, c2], counts=[2, 1])
    ws = [white_noise(32, 100), white_noise(32, 101), white_noise(16, 102)]
    p1, p2 = plan.displace(1.0, [to_dev(w, torch.float64) for w in ws])
    for w, q1, q2, cfg in zip(ws, p1, p2, (c1, c1, c2)):
        m = oracle_model(cfg)
        r1, r2 = fields.displace(w, m, 1.0, _tables(m, 1.0))
        assert normwise(q1, r1) < F64_TOL and normwise(q2, r2) < F64_TOL


def test_ticket_tile_order_repeats_exactly():
    # x tiles of 64-byte rows (and the fused y pass's 128-byte tiles) take
    # their tiles from per-XCD tickets, which every launch leaves at zero,
    # wherever a workgroup gets 8 tiles or more: at n = 256 with three
    # realisations the x passes have 3 x 4096 tiles of 8 columns for at most
    # 4 workgroups per CU, the fused y passes 3 x 2048 tiles for 2.  Three
    # calls in a row on one plan give the same bits, and the oracle's
    # displacements (the first and the last realisation of the shared tile
    # space)
    n = 256
    print(f"ticket tile order n={n}", flush=True)
    from paper_1909_06282_amd import Plan
    cfg = gpu_config(precision="fp32", n=n, box=2.0 * n, gravity="fr_hs", fr0_abs=1e-5, factorisation="t1",
                     nk_growth=64)
    plan = Plan(cfg, counts=[3])
    opts = plan.tile_options(0)
    plan.set_tiles(0, [0, 0, min(opts[2])])
    assert plan.get_tiles(0)[2] * 8 < 128 and plan.get_tiles(0)[1] * 8 >= 128
    ws = [white_noise(n, 21), white_noise(n, 22), white_noise(n, 23)]
    runs = []
    for _ in range(3):
        p1, p2 = plan.displace(1.0, [to_dev(w, torch.float32) for w in ws])
        runs.append([x.cpu() for x in p1 + p2])
    for r in runs[1:]:
        for a, b in zip(r, runs[0]):
            assert torch.equal(a, b)
    m = oracle_model(cfg)
    for k in (0, 2):
        r1, r2 = fields.displace(ws[k], m, 1.0, _tables(m, 1.0))
        e1, e2 = normwise(runs[0][k], r1), normwise(runs[0][3 + k], r2)
        print(f"  realisation {k}: psi1 {e1:.3e} psi2 {e2:.3e}", flush=True)
        assert e1 < F32_TOL and e2 < F32_TOL
    plan.close()


@pytest.mark.parametrize("prec", ["fp64", "fp32"])
def test_zero_noise_gives_zero_displacements(prec):
    # the degenerate input: every mode is zero, so are psi1, psi2 (exactly)
    print(f"zero noise {prec}", flush=True)
    plan, cfg = _plan(precision=prec, n=24, box=48.0, gravity="fr_hs", fr0_abs=1e-5, factorisation="t1",
                      nk_growth=64)
    w = torch.zeros((24, 24, 24), dtype=cfg.dtype, device="cuda")
    p1, p2 = plan.displace(1.0, w)
    torch.cuda.synchronize()
    assert not torch.any(p1) and not torch.any(p2)


def test_single_plane_wave_gives_no_psi2():
    print("plane wave", flush=True)
    plan, cfg = _plan(n=16, box=32.0, gravity="fr_hs", fr0_abs=1e-5, factorisation="t1", nk_growth=64)
    # white noise equal to one plane wave: its shaped delta is one Fourier mode
    c = np.arange(16)
    X, Y, Z = np.meshgrid(c, c, c, indexing="ij")
    w = np.cos(2 * np.pi * (X + 2 * Y - Z) / 16)
    p1, p2 = plan.displace(1.0, to_dev(w, torch.float64))
    assert float(p2.abs().max()) < 1e-13 * float(p1.abs().max())


@pytest.mark.parametrize("prec,tol", [("fp64", F64_TOL), ("fp32", F32_TOL)])
def test_displace_delta_matches_oracle(prec, tol):
    # a density field in place of white noise (no shaping): the oracle's
    # delta(k) path on F[delta]
    print(f"displace from delta(x) {prec}", flush=True)
    n = 32
    plan, cfg = _plan(precision=prec, n=n, box=64.0, gravity="fr_hs", fr0_abs=1e-5, factorisation="t1",
                      nk_growth=64)
    dx = 0.05 * white_noise(n, 11)
    p1, p2 = plan.displace_delta(0.8, to_dev(dx, cfg.dtype))
    torch.cuda.synchronize()
    m = oracle_model(cfg)
    dk = oracle.fft.rfftn(torch.from_numpy(dx))
    r1, r2 = fields.displace_from_delta_k(dk, m, 0.8, _tables(m, 0.8))
    e1, e2 = normwise(p1, r1), normwise(p2, r2)
    print(f"  psi1 {e1:.3e} psi2 {e2:.3e}", flush=True)
    assert e1 < tol and e2 < tol


def test_displace_delta_plane_wave_closed_form():
    # delta = A cos(k.x): psi1 = -A D1 k/k^2 sin(k.x) exactly and psi2 = 0
    print("displace from one plane wave", flush=True)
    n, box = 16, 32.0
    plan, cfg = _plan(n=n, box=box, gravity="gr", factorisation="eds")
    c = np.arange(n)
    X, Y, Z = np.meshgrid(c, c, c, indexing="ij")
    mvec = np.array([1, 2, -1])
    ph = 2 * np.pi * (mvec[0] * X + mvec[1] * Y + mvec[2] * Z) / n
    A = 0.01
    p1, p2 = plan.displace_delta(1.0, to_dev(A * np.cos(ph), torch.float64))
    _, d1, _ = plan.growth_table(1.0)
    kv = 2 * np.pi / box * mvec
    ref = np.stack([-A * d1[0] * kv[i] / (kv @ kv) * np.sin(ph) for i in range(3)])
    assert normwise(p1, ref) < 1e-12
    assert float(p2.abs().max()) < 1e-13 * float(p1.abs().max())


@pytest.mark.parametrize("prec", ["fp64", "fp32"])
def test_positions_match_oracle(prec):
    print(f"positions {prec}", flush=True)
    n = 32
    plan, cfg = _plan(precision=prec, n=n, box=64.0, gravity="fr_hs", fr0_abs=1e-5, factorisation="t1",
                      nk_growth=64)
    p1, p2 = plan.displace(1.0, to_dev(white_noise(n, 2), cfg.dtype))
    x = plan.positions(p1, p2)
    torch.cuda.synchronize()
    m = oracle_model(cfg)
    ref = fields.positions(p1.double().cpu(), p2.double().cpu(), m)
    d = (x.double().cpu() - ref).abs()
    d = torch.minimum(d, cfg.box - d)          # periodic distance
    tol = 1e-12 * cfg.box if prec == "fp64" else 1e-6 * cfg.box
    assert float(d.max()) < tol
    assert float(x.min()) >= 0.0 and float(x.max()) < cfg.box


@pytest.mark.parametrize("prec,tol", [("fp64", 1e-10), ("fp32", 1e-5)])
@pytest.mark.parametrize("deconvolve,interlace", [(False, False), (True, False), (False, True), (True, True)])
def test_matter_power_matches_oracle(prec, tol, deconvolve, interlace):
    # the same displacements on both sides: CIC paint(s), FFT, shells
    print(f"matter power {prec} deconvolve={deconvolve} interlace={interlace}", flush=True)
    n, nb = 32, 16
    plan, cfg = _plan(precision=prec, n=n, box=64.0, gravity="fr_hs", fr0_abs=1e-5, factorisation="t1",
                      nk_growth=64)
    p1, p2 = plan.displace(1.0, to_dev(white_noise(n, 4), cfg.dtype))
    got = plan.matter_power(p1, p2, nb, deconvolve, interlace=interlace)
    m = oracle_model(cfg)
    disp = p1.double().cpu() + p2.double().cpu()
    if interlace:
        km, cnt, mean, std = spectrum.matter_power_interlaced(disp, m, nb, deconvolve)
    else:
        km, cnt, mean, std = spectrum.matter_power(cic.paint(disp, m), m, nb, deconvolve)
    assert np.array_equal(got["count"], cnt)
    nz = cnt > 0
    err = np.max(np.abs(got["mean"][nz] / mean[nz] - 1))
    print(f"  max relative bin error {err:.3e}", flush=True)
    assert err < tol
    assert np.max(np.abs(got["k_mean"][nz] / km[nz] - 1)) < 1e-12


def test_auto_factorisation_plan():
    print("AUTO factorisation plan", flush=True)
    from paper_1909_06282_amd import LPT2Error, Plan
    n = 64
    kw = dict(n=n, box=256.0, gravity="fr_hs", fr0_abs=1e-4, nk_growth=64)
    plan, cfg = _plan(factorisation="auto", **kw)
    w = white_noise(n, 5)
    wd = to_dev(w, torch.float64)
    assert plan.auto_choice(0, 1.0) is None
    p1, p2 = plan.displace(1.0, wd)
    name = plan.auto_choice(0, 1.0)
    m = oracle_model(gpu_config(factorisation="t1", **kw))
    tab = _tables(m, 1.0)
    km, cnt, mean, _ = mgsource.source_ratio(w, m, 1.0, n // 2, tab)
    best, _ = mgsource.choose_triangle(km, cnt, mean, m, 1.0, 0.4, tab)
    print(f"  AUTO chose {name} (oracle {best})", flush=True)
    assert name == best
    from paper_1909_06282_amd import factorisation_candidate
    names = [factorisation_candidate(i)[0] for i in range(8)]
    _, r, th, win = factorisation_candidate(names.index(name))
    fk = dict(factorisation="winther") if win else (dict(factorisation="t1") if (r == 1.0 and th == 90.0) else
                                                    dict(factorisation="triangle", tri_ratio=r, tri_theta_deg=th))
    ref = Plan(gpu_config(**kw, **fk))
    q1, q2 = ref.displace(1.0, wd)
    torch.cuda.synchronize()
    assert torch.equal(p1, q1)
    assert normwise(p2, q2) < 1e-14     # T1 and a triangle at (1, 90) differ only in rounding
    with pytest.raises(LPT2Error):      # no choice at a = 0.5 yet
        plan.growth_table(0.5)
    with pytest.raises(LPT2Error):
        plan.displace_delta(0.5, wd)


# ---------------------------------------------------------------- source spectrum
@pytest.mark.parametrize("n,nbins", [(16, 8), (32, 16), (64, 32), (48, 24), (192, 96), (32, 1), (32, 512)])
def test_source_power_spectrum_matches_oracle(n, nbins):
    # nbins 1 and 512: the smallest and largest shell counts (512 shells of
    # width k_Nyq/512 on a 32^3 grid: most are empty and must count zero)
    print(f"source power n={n}", flush=True)
    plan, cfg = _plan(n=n, box=2.0 * n, gravity="fr_hs", fr0_abs=1e-5, factorisation="t1", nk_growth=64)
    w = white_noise(n, 3)
    got = plan.source_spectrum(1.0, to_dev(w, torch.float64), nbins, "power")
    m = oracle_model(cfg)
    sk = fields.source_k(fields.source(fields.delta_k(w, m), m), m)
    km, cnt, mean, std = spectrum.source_power(sk, m, nbins)
    assert np.array_equal(got["count"], cnt)
    nz = cnt > 0
    assert np.max(np.abs(got["k_mean"][nz] / km[nz] - 1)) < 1e-13
    assert np.max(np.abs(got["mean"][nz] / mean[nz] - 1)) < 1e-11
    sd = nz & (std > 1e-6 * np.abs(mean))
    assert np.max(np.abs(got["std"][sd] / std[sd] - 1)) < 1e-9
    # shells whose modes all have one value (e.g. a single mode): zero scatter
    flat = nz & ~sd
    assert np.all(np.abs(got["std"][flat]) <= 1e-6 * np.abs(mean[flat]) + 1e-300)


def test_source_spectrum_is_bitwise_reproducible():
    print("binner determinism", flush=True)
    plan, cfg = _plan(precision="fp32", n=64, box=128.0, gravity="fr_hs", fr0_abs=1e-5, factorisation="t1",
                      nk_growth=64)
    w = to_dev(white_noise(64, 9), torch.float32)
    a = plan.source_spectrum(1.0, w, 32, "power")
    b = plan.source_spectrum(1.0, w, 32, "power")
    for k in a:
        assert np.array_equal(a[k], b[k])


@pytest.mark.parametrize("gravity", ["gr", "fr_hs"])
def test_source_ratio_matches_oracle(gravity):
    print(f"source ratio {gravity}", flush=True)
    n, nb = 32, 16
    plan, cfg = _plan(n=n, box=128.0, gravity=gravity, fr0_abs=1e-4, factorisation="t1", nk_growth=64)
    w = white_noise(n, 3)
    got = plan.source_spectrum(1.0, to_dev(w, torch.float64), nb, "ratio")
    m = oracle_model(cfg)
    km, cnt, mean, std = mgsource.source_ratio(w, m, 1.0, nb, _tables(m, 1.0))
    assert np.array_equal(got["count"], cnt)
    nz = cnt > 0
    assert np.max(np.abs(got["mean"][nz] - mean[nz])) < 1e-10
    assert np.max(np.abs(got["std"][nz] - std[nz])) < 1e-7
    if gravity == "gr":
        assert np.max(np.abs(got["mean"][nz] - 1)) < 1e-12


def test_choose_factorisation_matches_oracle():
    print("factorisation choice f(R) 64^3", flush=True)
    from paper_1909_06282_amd import LPT2Error, Plan
    n, nb = 64, 32
    plan, cfg = _plan(n=n, box=256.0, gravity="fr_hs", fr0_abs=1e-4, factorisation="eds", nk_growth=64)
    w = white_noise(n, 5)
    wd = to_dev(w, torch.float64)
    name, costs = plan.choose_factorisation(1.0, wd, nbins=nb, kcut=0.4)
    m = oracle_model(cfg)
    tab = _tables(m, 1.0)
    km, cnt, mean, _ = mgsource.source_ratio(w, m, 1.0, nb, tab)
    best, ocosts = mgsource.choose_triangle(km, cnt, mean, m, 1.0, 0.4, tab)
    print(f"  chosen {name} (oracle {best}); costs {costs}", flush=True)
    assert name == best
    assert set(costs) == set(ocosts)
    for k, v in ocosts.items():
        assert abs(costs[k] - v) <= 1e-8 * max(1.0, abs(v)), k
    # apply: the plan's D2 table becomes the chosen candidate's
    name2, _ = plan.choose_factorisation(1.0, wd, nbins=nb, kcut=0.4, apply=True)
    assert name2 == name
    p1, p2 = plan.displace(1.0, wd)
    from paper_1909_06282_amd import factorisation_candidate
    _, r, th, win = factorisation_candidate(list(costs).index(name))
    kw = dict(factorisation="winther") if win else (dict(factorisation="t1") if (r == 1.0 and th == 90.0) else
                                                    dict(factorisation="triangle", tri_ratio=r, tri_theta_deg=th))
    ref = Plan(gpu_config(n=n, box=256.0, gravity="fr_hs", fr0_abs=1e-4, nk_growth=64, **kw))
    q1, q2 = ref.displace(1.0, wd)
    torch.cuda.synchronize()
    assert torch.equal(p1, q1) and torch.equal(p2, q2)
    with pytest.raises(LPT2Error):
        plan.choose_factorisation(1.0, wd, nbins=nb, kcut=1e-4)


def test_triangle_ratio_matches_oracle():
    plan, cfg = _plan(n=8, box=16.0, gravity="fr_hs", fr0_abs=1e-4, factorisation="t1", nk_growth=64)
    m = oracle_model(cfg)
    k = np.geomspace(0.01, 1.0, 9)
    tab = growth.tables(m.with_(factorisation="eds"), 0.8)
    for _, r, th, win in mgsource.CANDIDATES:
        got = plan.triangle_ratio(0.8, r, th, k, win)
        ref = mgsource.triangle_ratio(k, m, 0.8, r, th, win, tab)
        assert np.max(np.abs(got / ref - 1)) < 1e-12, (r, th, win)


# ---------------------------------------------------------------- adjoint and CIC
@pytest.mark.parametrize("n", [8, 16, 40, 48, 56, 64, 96])
def test_backward_matches_oracle_autograd(n):
    # 64: the x passes' paired radial gathers (last radix 8) are on; 40, 56:
    # transforms with a factor 5 or 7 (the LDS-staged engine)
    print(f"backward fp64 n={n}", flush=True)
    plan, cfg = _plan(n=n, box=2.0 * n, gravity="fr_hs", fr0_abs=1e-5, factorisation="t1", nk_growth=64)
    m = oracle_model(cfg)
    w = white_noise(n, 4)
    rng = np.random.default_rng(5)
    g1, g2 = rng.standard_normal((3, n, n, n)), rng.standard_normal((3, n, n, n))
    got = plan.backward(1.0, to_dev(w, torch.float64), to_dev(g1, torch.float64), to_dev(g2, torch.float64))
    ref = adjoint.vjp_displace(w, g1, g2, m, 1.0, _tables(m, 1.0))
    assert normwise(got, ref) < 1e-11


@pytest.mark.parametrize("n", [32, 40, 48, 56, 64])
def test_backward_fp32_matches_fp64_gpu(n):
    print(f"backward fp32 n={n}", flush=True)
    kw = dict(n=n, box=2.0 * n, gravity="fr_hs", fr0_abs=1e-5, factorisation="t1", nk_growth=64)
    p64, _ = _plan(precision="fp64", **kw)
    p32, _ = _plan(precision="fp32", **kw)
    w = white_noise(n, 4)
    rng = np.random.default_rng(6)
    g1, g2 = rng.standard_normal((3, n, n, n)), rng.standard_normal((3, n, n, n))
    a = p64.backward(1.0, to_dev(w, torch.float64), to_dev(g1, torch.float64), to_dev(g2, torch.float64))
    b = p32.backward(1.0, to_dev(w, torch.float32), to_dev(g1, torch.float32), to_dev(g2, torch.float32))
    assert normwise(b, a) < F32_TOL


@pytest.mark.parametrize("n,stretch", [(16, 1.0), (8, 1.0), (24, 1.0), (48, 1.0), (32, 6.0)])
def test_cic_paint_and_transpose_match_oracle(n, stretch):
    # n = 8: one tile per axis (both regions covering a cell are the same
    # tile); 24, 48: an odd number of tiles; stretch 6: most particles leave
    # their tile's halo and are added with atomics
    print(f"cic n={n} stretch={stretch}", flush=True)
    plan, cfg = _plan(n=n, box=2.0 * n, gravity="fr_hs", fr0_abs=1e-5, factorisation="t1", nk_growth=64)
    m = oracle_model(cfg)
    w = white_noise(n, 7)
    p1, p2 = plan.displace(1.0, to_dev(w, torch.float64))
    p1, p2 = p1 * stretch, p2 * stretch
    d = plan.paint_cic(p1, p2)
    ref = cic.paint(p1.cpu() + p2.cpu(), m)
    assert float((d.cpu() - ref).abs().max()) < 1e-12
    gd = np.random.default_rng(8).standard_normal((n, n, n))
    g = plan.paint_cic_backward(p1, p2, to_dev(gd, torch.float64))
    gref = adjoint.vjp_paint(p1.cpu() + p2.cpu(), gd, m)
    assert normwise(g, gref) < 1e-12


@pytest.mark.parametrize("prec", ["fp64", "fp32"])
def test_check_finite_counts_nonfinite_noise(prec):
    # the displacement entry points do not scan their inputs; lpt2_check_finite
    # finds the non-finite values of a noise field before it is used
    print(f"check_finite {prec}", flush=True)
    from paper_1909_06282_amd import _abi
    plan, cfg = _plan(precision=prec, n=32, box=64.0)
    w = to_dev(white_noise(32, 1), cfg.dtype)
    assert plan.check_finite(w) == 0
    flat = w.view(-1)
    flat[5] = float("nan")
    flat[32 ** 3 - 1] = float("inf")
    flat[1000] = -float("inf")
    assert plan.check_finite(w) == 3
    import ctypes as C
    L = _abi.load()
    cnt = C.c_longlong()
    st = L.lpt2_check_finite(plan.handle, C.c_void_p(w.data_ptr()), w.numel(), C.byref(cnt), None)
    assert st == _abi.EINVAL and cnt.value == 3
    assert b"non-finite" in L.lpt2_last_error(plan.handle)
    plan.close()


def test_allocation_failures_return_enomem_and_leave_no_state(monkeypatch):
    # LPT2_FAIL_ALLOC=k fails the k-th device allocation after lpt2_plan
    # starts: the plan's own allocations (twiddles, workspace, binner), then
    # the growth tables of the first displacement; each gives LPT2_ENOMEM,
    # releases what was allocated, and a plan made afterwards works
    print("allocation failure injection", flush=True)
    from paper_1909_06282_amd import LPT2Error, _abi
    kw = dict(precision="fp64", n=16, box=32.0, gravity="fr_hs", fr0_abs=1e-5, factorisation="t1", nk_growth=32)
    w = to_dev(white_noise(16, 2), torch.float64)
    for k in (1, 2, 3):
        monkeypatch.setenv("LPT2_FAIL_ALLOC", str(k))
        with pytest.raises(LPT2Error) as ei:
            _plan(**kw)
        assert ei.value.status == _abi.ENOMEM, (k, str(ei.value))
    for k in (4, 5):                     # growth table, then radial table of the first call at a
        monkeypatch.setenv("LPT2_FAIL_ALLOC", str(k))
        plan, cfg = _plan(**kw)
        with pytest.raises(LPT2Error) as ei:
            plan.displace(1.0, w)
        assert ei.value.status == _abi.ENOMEM, (k, str(ei.value))
        plan.close()
    monkeypatch.delenv("LPT2_FAIL_ALLOC")
    plan, cfg = _plan(**kw)
    p1, p2 = plan.displace(1.0, w)
    torch.cuda.synchronize()
    m = oracle_model(cfg)
    r1, r2 = fields.displace(white_noise(16, 2), m, 1.0, _tables(m, 1.0))
    assert normwise(p1, r1) < F64_TOL and normwise(p2, r2) < F64_TOL
    plan.close()


def test_invalid_arguments_raise():
    from paper_1909_06282_amd import LPT2Error
    plan, cfg = _plan(n=8, box=16.0)
    w = to_dev(white_noise(8, 1), torch.float64)
    with pytest.raises(LPT2Error):
        plan.displace(0.0, w)
    with pytest.raises(LPT2Error):
        plan.displace(-1.0, w)
    with pytest.raises(ValueError):
        plan.displace(1.0, w.float())
    with pytest.raises(ValueError):
        plan.displace(1.0, to_dev(white_noise(16, 1), torch.float64))
    # matter power: a flag bit that is not defined
    import ctypes
    from paper_1909_06282_amd import _abi
    p1, p2 = plan.displace(1.0, w)
    out = [np.zeros(4) for _ in range(4)]
    ptr = [o.ctypes.data_as(ctypes.POINTER(ctypes.c_double)) for o in out]
    st = plan._lib.lpt2_matter_power(plan.handle, ctypes.c_void_p(p1.data_ptr()), ctypes.c_void_p(p2.data_ptr()), 4,
                                     4, *ptr, None)
    assert st == _abi.EINVAL
