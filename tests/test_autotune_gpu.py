"""Tunables of the plans and the autotuner: every setting of the tunables
(leaf-tile splits, work cap of leaf items, weight of surface sources, GEMM
row blocks per wave, the order of the pair evaluation's passes) gives the same FMM within rounding (single precision
against the default setting 1e-6, and the FP64 direct sum 1e-4); the
autotuner returns a setting from its candidate lists that meets the same
bar, and caches it."""
import json

import numpy as np
import pytest

import synth
from oracle import direct as D
from tests.gpu_util import require_gpu

pytestmark = pytest.mark.gpu
KAPPA = 0.125


def _cloud():
    su = synth.sphere_union_spheres(30, seed=131, box=14.0)
    v, t = synth.sphere_union_mesh(su, 6000, seed=131)
    return synth.three_point_cloud(v, t)


def _pair(xt, q, ncrit=48):
    from paper_2103_01048_amd import FMMPlan, eval_pair
    a = FMMPlan(xt, kernel="laplace", p=6, ncrit=ncrit, precision="bf16x3")
    b = FMMPlan(xt, kernel="yukawa", kappa=KAPPA, p=6, ncrit=ncrit, precision="bf16x3")
    (pa, ga), (pb, gb) = eval_pair(a, b, q)
    return [t.double().cpu().numpy() for t in (pa, ga, pb, gb)]


@pytest.mark.parametrize("setting", [
    {"tile_split2": 0, "tile_split4": 0},
    {"tile_split2": 24, "tile_split4": 12},
    {"work_cap_div": 262144, "work_cap_min": 64},
    {"work_cap_div": 256},
    {"far_weight": 3.0},
    {"gemm_rbw": 1},
    {"gemm_rbw": 4},
    {"pair_order": 1},
    {"pair_order": 2},
    {"pair_order": 3},
    {"gemm_lat": 0},
    {"gemm_lat": 1 << 20},
    {"near_lds": 13312},
    {"m2l_cols": 128},
    {"gemm_narrow": 1},
    {"gemm_narrow": 1, "pair_order": 3},
    {"near_early": 300},
    {"near_early": 900, "near_early_grid": 64},
    {"m2l_early": 1},
    {"m2l_early": 1, "near_early": 500, "gemm_narrow": 1},
    {"near_early": 450, "near_early_start": 1},
    {"pair_order": 4},
    {"pair_order": 4, "near_early": 400, "near_early_start": 1, "gemm_narrow": 1, "m2l_early": 1},
    {"pair_order": 4, "near_early": 300},
])
def test_every_setting_gives_the_same_fmm(setting):
    torch = require_gpu()
    from paper_2103_01048_amd import autotune as at
    x = _cloud()
    q = np.random.default_rng(132).standard_normal(len(x))
    xt = torch.tensor(x, device="cuda")
    qt = torch.tensor(q, device="cuda", dtype=torch.float32)
    print(f"[tuning] {setting}", flush=True)
    ref = _pair(xt, qt)
    with at.tuning(**setting):
        got = _pair(xt, qt)
    for r, g in zip(ref, got):
        assert np.linalg.norm(g - r) / np.linalg.norm(r) < 1e-6
    rows = np.arange(0, len(x), 7)
    for k, (pot, grad) in (("laplace", got[:2]), ("yukawa", got[2:])):
        p0, g0 = D.direct(x[rows], x, q, k, KAPPA)
        assert D.rel_l2(pot[rows], p0) < 1e-4 and D.rel_l2(grad[rows], g0) < 1e-4


def test_autotune_picks_a_candidate_and_caches_it(tmp_path):
    torch = require_gpu()
    from paper_2103_01048_amd import autotune as at
    x = _cloud()
    xt = torch.tensor(x, device="cuda")
    cache = str(tmp_path / "tuning.json")
    before = at.get_tuning()
    res = at.autotune(xt, p=6, ncrit_candidates=(32, 64), steps=2, warmup=1, cache_path=cache)
    print(f"[autotune] {res['ncrit']} {res['tuning']} {res['ms']} ms, {len(res['trials'])} trials", flush=True)
    assert at.get_tuning() == before
    assert res["ncrit"] in (32, 64) and not res["cached"]
    assert len(res["trials"]) >= 2 + 3
    stored = json.load(open(cache))
    assert stored[res["key"]]["ncrit"] == res["ncrit"]
    again = at.autotune(xt, p=6, ncrit_candidates=(32, 64), cache_path=cache)
    assert again["cached"] and again["tuning"] == res["tuning"]
    ncrit = at.apply(res)
    try:
        q = np.random.default_rng(133).standard_normal(len(x))
        pa, ga, pb, gb = _pair(xt, torch.tensor(q, device="cuda", dtype=torch.float32), ncrit=ncrit)
        rows = np.arange(0, len(x), 7)
        p0, g0 = D.direct(x[rows], x, q, "yukawa", KAPPA)
        assert D.rel_l2(pb[rows], p0) < 1e-4 and D.rel_l2(gb[rows], g0) < 1e-4
    finally:
        at.set_tuning(**before)


@pytest.mark.parametrize("precision,tol,tol_dense", [("bf16x3", 1e-4, 1e-5), ("fp32", 1e-4, 1e-5),
                                                      ("fp64", 1e-6, 1e-9)])
def test_factored_m2l(precision, tol, tol_dense):
    """M2L with each offset's operator split by its own truncated SVD
    (m2l_factored): against the direct sum at the precision's bar and against
    the dense M2L within the truncation, for the pair evaluation and for one
    plan alone."""
    torch = require_gpu()
    from paper_2103_01048_amd import FMMPlan, autotune as at, eval_pair
    x = _cloud()
    q = np.random.default_rng(134).standard_normal(len(x))
    xt = torch.tensor(x, device="cuda")
    qt = torch.tensor(q, device="cuda", dtype=torch.float64 if precision == "fp64" else torch.float32)
    mk = lambda k: FMMPlan(xt, kernel=k, kappa=KAPPA, p=8, ncrit=48, precision=precision)
    dense = [mk("laplace"), mk("yukawa")]
    with at.tuning(m2l_factored=1):
        fact = [mk("laplace"), mk("yukawa")]
    print(f"[factored m2l] {precision}", flush=True)
    outs_d = eval_pair(dense[0], dense[1], qt)
    outs_f = eval_pair(fact[0], fact[1], qt)
    alone = fact[1].eval(qt)
    rows = np.arange(0, len(x), 5)
    for k, od, of in zip(("laplace", "yukawa"), outs_d, outs_f):
        p0, g0 = D.direct(x[rows], x, q, k, KAPPA)
        pf, gf = of[0].double().cpu().numpy(), of[1].double().cpu().numpy()
        pd, gd = od[0].double().cpu().numpy(), od[1].double().cpu().numpy()
        print(f"  {k}: direct pot {D.rel_l2(pf[rows], p0):.2e} grad {D.rel_l2(gf[rows], g0):.2e}; "
              f"dense pot {D.rel_l2(pf, pd):.2e} grad {D.rel_l2(gf, gd):.2e}", flush=True)
        assert D.rel_l2(pf[rows], p0) < tol and D.rel_l2(gf[rows], g0) < tol
        assert D.rel_l2(pf, pd) < tol_dense and D.rel_l2(gf, gd) < tol_dense
    assert D.rel_l2(alone[0].double().cpu().numpy(), outs_f[1][0].double().cpu().numpy()) < 1e-6


@pytest.mark.parametrize("precision,p", [("bf16x3", 6), ("fp32", 8), ("fp64", 4)])
def test_chained_level_launches_equal_per_level_launches(precision, p):
    """The M2M levels and the L2L levels of a pair evaluation in one chained
    launch each (gemm_chain): the same GEMM tiles and sums in the same order
    as one launch per level, so the results are equal bit for bit, on every
    repeat; no chained wait hits its bound."""
    torch = require_gpu()
    from paper_2103_01048_amd import FMMPlan, autotune as at, eval_pair
    x = _cloud()
    q = np.random.default_rng(135).standard_normal(len(x))
    xt = torch.tensor(x, device="cuda")
    qt = torch.tensor(q, device="cuda", dtype=torch.float64 if precision == "fp64" else torch.float32)
    mk = lambda k: FMMPlan(xt, kernel=k, kappa=KAPPA, p=p, ncrit=32, precision=precision)
    per_level = [mk("laplace"), mk("yukawa")]
    with at.tuning(gemm_chain=1):
        chained = [mk("laplace"), mk("yukawa")]
    print(f"[chain] {precision} p={p} levels {per_level[0].info()['max_level']}", flush=True)
    ref = [t.cpu().numpy() for o in eval_pair(per_level[0], per_level[1], qt) for t in o]
    for _ in range(3):
        got = [t.cpu().numpy() for o in eval_pair(chained[0], chained[1], qt) for t in o]
        for r, g in zip(ref, got):
            assert np.array_equal(r, g)
    assert chained[0].info()["chain_timeouts"] == 0
    # one launch each for the M2M and the L2L levels (the per-level path has
    # one per level)
    for pls, one in ((chained, True), (per_level, False)):
        pls[0].set_profiling(True)
        pls[0].phase_times()
        eval_pair(pls[0], pls[1], qt)
        ph = pls[0].phase_times()
        pls[0].set_profiling(False)
        assert (ph["m2m"][1] == 1 and ph["l2l"][1] == 1) == one, ph


@pytest.mark.parametrize("near_early", [0, 500])
def test_timed_near_launch_leaves_results_unchanged(near_early):
    """Timing the near field (its launches carry the timing events) counts
    one timed main launch per pair evaluation and, when the shortest items
    start early, one early launch under a phase of its own; the durations
    are positive and the results equal an untimed evaluation bit for bit.
    fmm_info splits the items and their pair interactions between the two
    launches."""
    torch = require_gpu()
    from paper_2103_01048_amd import FMMPlan, autotune as at, eval_pair
    x = _cloud()
    q = np.random.default_rng(137).standard_normal(len(x))
    xt = torch.tensor(x, device="cuda")
    qt = torch.tensor(q, device="cuda", dtype=torch.float32)
    with at.tuning(near_early=near_early):
        a = FMMPlan(xt, kernel="laplace", p=6, ncrit=48, precision="bf16x3")
        b = FMMPlan(xt, kernel="yukawa", kappa=KAPPA, p=6, ncrit=48, precision="bf16x3")
    inf = a.info()
    assert inf["max_level"] >= 2 and inf["n_items"] > 0
    assert inf["n_items_early"] == inf["n_items"] * near_early // 1000
    if near_early:
        assert 0 < inf["n_p2p_early"] < inf["n_p2p_interactions"]
    else:
        assert inf["n_p2p_early"] == 0
    ref = [t.cpu().numpy() for o in eval_pair(a, b, qt) for t in o]
    a.set_profiling(["near", "near_early"])
    a.phase_times()
    for _ in range(3):
        got = [t.cpu().numpy() for o in eval_pair(a, b, qt) for t in o]
        for r, g in zip(ref, got):
            assert np.array_equal(r, g)
    ph = a.phase_times()
    a.set_profiling(False)
    assert ph["near"][1] == 3 and ph["near"][0] > 0.0, ph
    assert ph["near_early"][1] == (3 if near_early else 0), ph
    assert (ph["near_early"][0] > 0.0) == bool(near_early), ph
    assert all(c == 0 for k, (_, c) in ph.items() if k not in ("near", "near_early")), ph
