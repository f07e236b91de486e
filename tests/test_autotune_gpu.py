"""Tunables of the plans and the autotuner: every setting of the tunables
(leaf-tile splits, work cap of leaf items, weight of surface sources, GEMM
row blocks per wave) gives the same FMM within rounding (single precision
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
