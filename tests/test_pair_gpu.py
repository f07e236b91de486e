"""fmm_eval_pair: a Laplace and a Yukawa plan on one tree evaluated together
(far-field passes on two side streams, one near-field launch for both
kernels) give the results of two fmm_eval calls, and match the FP64 direct
sum."""
import numpy as np
import pytest

import synth
from oracle import direct as D
from tests.gpu_util import require_gpu

pytestmark = pytest.mark.gpu
KAPPA = 0.125


def _cloud(n_tri=4000, seed=111):
    su = synth.sphere_union_spheres(30, seed=seed, box=14.0)
    v, t = synth.sphere_union_mesh(su, n_tri, seed=seed)
    return synth.three_point_cloud(v, t)


def _plans(x, precision, ncrit=64, offsets=None, ncrit_b=None):
    torch = require_gpu()
    from paper_2103_01048_amd import FMMPlan
    xt = torch.tensor(x, device="cuda")
    a = FMMPlan(xt, kernel="laplace", p=6, ncrit=ncrit, precision=precision, offsets=offsets)
    b = FMMPlan(xt, kernel="yukawa", kappa=KAPPA, p=6, ncrit=ncrit_b or ncrit, precision=precision, offsets=offsets)
    return a, b


def _rel(a, b):
    a = a.double().cpu().numpy()
    b = b.double().cpu().numpy()
    return float(np.linalg.norm(a - b) / np.linalg.norm(b))


@pytest.mark.parametrize("precision,tol", [("fp64", 1e-12), ("fp32", 1e-6), ("bf16x3", 1e-6)])
@pytest.mark.parametrize("nrhs", [1, 4])
def test_pair_equals_two_evals(precision, tol, nrhs):
    torch = require_gpu()
    from paper_2103_01048_amd import eval_pair
    x = _cloud()
    a, b = _plans(x, precision)
    q = torch.tensor(np.random.default_rng(112).standard_normal((nrhs, len(x))), device="cuda").to(a.dtype)
    (pa, ga), (pb, gb) = eval_pair(a, b, q)
    ra, rga = a.eval(q)
    rb, rgb = b.eval(q)
    errs = [_rel(pa, ra), _rel(ga, rga), _rel(pb, rb), _rel(gb, rgb)]
    print(f"[pair {precision} nrhs {nrhs}] {errs}", flush=True)
    assert max(errs) < tol


def test_pair_matches_direct_sum_and_is_deterministic():
    torch = require_gpu()
    from paper_2103_01048_amd import eval_pair
    x = _cloud(3000, seed=113)
    q = np.random.default_rng(113).standard_normal(len(x))
    a, b = _plans(x, "fp32")
    qt = torch.tensor(q, device="cuda", dtype=torch.float32)
    (pa, ga), (pb, gb) = eval_pair(a, b, qt)
    (pa2, ga2), (pb2, gb2) = eval_pair(a, b, qt)
    for u, w in ((pa, pa2), (ga, ga2), (pb, pb2), (gb, gb2)):
        assert torch.equal(u, w)
    for (pot, grad), kern, kap in (((pa, ga), "laplace", 0.0), ((pb, gb), "yukawa", KAPPA)):
        phi, g = D.direct(x, x, q, kern, kap)
        ep = D.rel_l2(pot.double().cpu().numpy(), phi)
        eg = D.rel_l2(grad.double().cpu().numpy(), g)
        print(f"[pair vs direct {kern}] pot {ep:.2e} grad {eg:.2e}", flush=True)
        assert ep < 1e-4 and eg < 1e-4


def test_pair_without_gradient_and_batched():
    torch = require_gpu()
    from paper_2103_01048_amd import eval_pair
    xs = [_cloud(1500, seed=114 + k) + 40.0 * k for k in range(3)]
    off = np.concatenate([[0], np.cumsum([len(x) for x in xs])])
    X = np.concatenate(xs)
    a, b = _plans(X, "fp32", offsets=off)
    q = torch.tensor(np.random.default_rng(117).standard_normal(len(X)), device="cuda", dtype=torch.float32)
    (pa, ga), (pb, gb) = eval_pair(a, b, q, gradient=False)
    assert ga is None and gb is None
    assert _rel(pa, a.eval(q, gradient=False)[0]) < 1e-6
    assert _rel(pb, b.eval(q, gradient=False)[0]) < 1e-6


def test_pair_on_different_trees_runs_one_after_the_other():
    """Plans with different ncrit do not share a tree: the pair call falls
    back to two evaluations and still returns both results."""
    torch = require_gpu()
    from paper_2103_01048_amd import eval_pair
    x = _cloud(2000, seed=118)
    a, b = _plans(x, "fp32", ncrit=64, ncrit_b=32)
    q = torch.tensor(np.random.default_rng(118).standard_normal(len(x)), device="cuda", dtype=torch.float32)
    (pa, ga), (pb, gb) = eval_pair(a, b, q)
    assert torch.equal(pa, a.eval(q)[0]) and torch.equal(pb, b.eval(q)[0])


def test_pair_rejects_mismatched_plans():
    torch = require_gpu()
    from paper_2103_01048_amd import FMMPlan, eval_pair
    x = _cloud(1000, seed=119)
    a = FMMPlan(torch.tensor(x, device="cuda"), kernel="laplace", p=4, ncrit=64, precision="fp32")
    b = FMMPlan(torch.tensor(x[:-3], device="cuda"), kernel="yukawa", kappa=KAPPA, p=4, ncrit=64, precision="fp32")
    q = torch.zeros(len(x), device="cuda")
    with pytest.raises(ValueError):
        eval_pair(a, b, q)


def _md_reference(x, q, dip, kern, kap, cq):
    """sum_j [cq q_j g + dip_j . grad_y g] from the oracle's N-body sum:
    grad_y g(x, y) = -grad_x g(x, y), so the dipole part is minus the
    divergence-like sum of the target gradients of the three dipole columns."""
    phi, _ = D.direct(x, x, q, kern, kap)
    out = cq * phi
    for d in range(3):
        _, g = D.direct(x, x, dip[:, d], kern, kap)
        out -= g[:, d]
    return out


@pytest.mark.parametrize("precision,tol", [("fp64", 1e-6), ("fp32", 1e-4), ("bf16x3", 1e-4)])
def test_pair_monopole_dipole_matches_direct_sum(precision, tol):
    torch = require_gpu()
    from paper_2103_01048_amd import FMMPlan, eval_pair_md
    x = _cloud(3000, seed=121)
    rng = np.random.default_rng(121)
    q = rng.standard_normal(len(x))
    dip = rng.standard_normal((len(x), 3))
    xt = torch.tensor(x, device="cuda")
    a = FMMPlan(xt, kernel="laplace", p=8, ncrit=64, precision=precision)
    b = FMMPlan(xt, kernel="yukawa", kappa=KAPPA, p=8, ncrit=64, precision=precision)
    pa, pb = eval_pair_md(a, b, torch.tensor(q, device="cuda"), torch.tensor(dip, device="cuda"), -1.0, -0.05)
    ra = _md_reference(x, q, dip, "laplace", 0.0, -1.0)
    rb = _md_reference(x, q, dip, "yukawa", KAPPA, -0.05)
    ea = D.rel_l2(pa.double().cpu().numpy(), ra)
    eb = D.rel_l2(pb.double().cpu().numpy(), rb)
    print(f"[pair md {precision}] laplace {ea:.2e} yukawa {eb:.2e}", flush=True)
    assert ea < tol and eb < tol


def test_pair_monopole_dipole_without_dipoles_equals_pair_potential():
    torch = require_gpu()
    from paper_2103_01048_amd import eval_pair, eval_pair_md
    x = _cloud(2000, seed=122)
    a, b = _plans(x, "fp64")
    q = torch.tensor(np.random.default_rng(122).standard_normal(len(x)), device="cuda")
    pa, pb = eval_pair_md(a, b, q, torch.zeros((len(x), 3), device="cuda", dtype=torch.float64), 2.0, 3.0)
    (ra, _), (rb, _) = eval_pair(a, b, q, gradient=False)
    assert _rel(pa, 2.0 * ra) < 1e-13 and _rel(pb, 3.0 * rb) < 1e-13


def test_pair_monopole_dipole_rejects_plans_without_a_shared_tree():
    torch = require_gpu()
    from paper_2103_01048_amd import FmmError, eval_pair_md
    x = _cloud(1500, seed=123)
    a, b = _plans(x, "fp32", ncrit=64, ncrit_b=32)
    with pytest.raises(FmmError):
        eval_pair_md(a, b, torch.zeros(len(x), device="cuda"), torch.zeros((len(x), 3), device="cuda"))


def test_pair_monopole_dipole_gradient_against_finite_differences():
    """grad_x of the monopole + dipole potential (FP64 path) at 48 sampled
    points against central differences (h = 1e-5 A) of the oracle's sums at
    shifted targets (the point's own source left out)."""
    torch = require_gpu()
    from paper_2103_01048_amd import FMMPlan, eval_pair_md
    x = _cloud(2500, seed=124)
    rng = np.random.default_rng(124)
    q = rng.standard_normal(len(x))
    dip = rng.standard_normal((len(x), 3))
    xt = torch.tensor(x, device="cuda")
    a = FMMPlan(xt, kernel="laplace", p=10, ncrit=64, precision="fp64")
    b = FMMPlan(xt, kernel="yukawa", kappa=KAPPA, p=10, ncrit=64, precision="fp64")
    (pa, ga), (pb, gb) = eval_pair_md(a, b, torch.tensor(q, device="cuda"), torch.tensor(dip, device="cuda"),
                                      -1.0, -0.05, gradient=True)
    ga, gb = ga.cpu().numpy(), gb.cpu().numpy()
    pick = rng.choice(len(x), 48, replace=False)
    h = 1e-5
    for kern, kap, cq, g in (("laplace", 0.0, -1.0, ga), ("yukawa", KAPPA, -0.05, gb)):
        fd = np.zeros((48, 3))
        for i, k in enumerate(pick):
            keep = np.delete(np.arange(len(x)), k)
            for d in range(3):
                e = np.zeros(3)
                e[d] = h
                pts = np.stack([x[k] + e, x[k] - e])
                vals = _md_reference_at(pts, x[keep], q[keep], dip[keep], kern, kap, cq)
                fd[i, d] = (vals[0] - vals[1]) / (2 * h)
        err = D.rel_l2(g[pick], fd)
        print(f"[md gradient {kern}] rel {err:.2e}", flush=True)
        assert err < 1e-6


def _md_reference_at(tx, sx, q, dip, kern, kap, cq):
    phi, _ = D.direct(tx, sx, q, kern, kap)
    out = cq * phi
    for d in range(3):
        _, g = D.direct(tx, sx, dip[:, d], kern, kap)
        out -= g[:, d]
    return out


@pytest.mark.parametrize("how", ["scaled", "moved"])
def test_plans_on_other_points_do_not_share_a_tree(how):
    """A Yukawa plan on 1.5 x (same tree topology, other geometry) or on
    slightly moved points (same topology and root cube) must not share the
    Laplace plan's tree: fmm_eval_pair then gives the two fmm_eval results."""
    torch = require_gpu()
    from paper_2103_01048_amd import FMMPlan, eval_pair
    x = _cloud(2000, seed=117)
    if how == "scaled":
        x2 = 1.5 * x
    else:
        x2 = x.copy()
        x2[:, 0] += 1e-7 * np.random.default_rng(117).standard_normal(len(x))
    xa = torch.tensor(x, device="cuda")
    xb = torch.tensor(x2, device="cuda")
    for prec in ("fp64", "fp32"):
        a = FMMPlan(xa, kernel="laplace", p=5, ncrit=64, precision=prec)
        b = FMMPlan(xb, kernel="yukawa", kappa=KAPPA, p=5, ncrit=64, precision=prec)
        q = torch.tensor(np.random.default_rng(118).standard_normal(len(x)), device="cuda").to(a.dtype)
        (pa, ga), (pb, gb) = eval_pair(a, b, q)
        ra, rga = a.eval(q)
        rb, rgb = b.eval(q)
        errs = [_rel(pa, ra), _rel(ga, rga), _rel(pb, rb), _rel(gb, rgb)]
        print(f"[pair on other points, {how} {prec}] {errs}", flush=True)
        assert max(errs) == 0.0


def test_second_plan_shares_the_tree_and_outlives_the_first():
    """A Yukawa plan built while a Laplace plan on the same points (same
    ncrit, p, working type) is alive takes that plan's tree, lists and leaf
    items (fmm_info: tree_shared); freeing the Laplace plan leaves the Yukawa
    plan's results unchanged.  Plans on other points, or with another ncrit,
    build their own tree on the device."""
    torch = require_gpu()
    import gc
    from paper_2103_01048_amd import FMMPlan
    x = _cloud(3000, seed=119)
    xt = torch.tensor(x, device="cuda")
    q = torch.tensor(np.random.default_rng(119).standard_normal(len(x)), device="cuda", dtype=torch.float32)
    a = FMMPlan(xt, kernel="laplace", p=6, ncrit=64, precision="bf16x3")
    b = FMMPlan(xt, kernel="yukawa", kappa=KAPPA, p=6, ncrit=64, precision="bf16x3")
    ia, ib = a.info(), b.info()
    assert ia["tree_on_device"] == 1 and ia["tree_shared"] == 0
    assert ib["tree_shared"] == 1 and ib["n_boxes"] == ia["n_boxes"]
    ta, tb = a.tree(), b.tree()
    for k in ("perm", "keys", "level", "anchor", "begin", "end", "list_off", "list_idx"):
        assert np.array_equal(ta[k], tb[k]), k
    pb0, gb0 = b.eval(q)
    torch.cuda.synchronize()
    pb0, gb0 = pb0.clone(), gb0.clone()
    del a
    gc.collect()
    pb1, gb1 = b.eval(q)
    torch.cuda.synchronize()
    assert torch.equal(pb0, pb1) and torch.equal(gb0, gb1)
    c = FMMPlan(xt, kernel="yukawa", kappa=KAPPA, p=6, ncrit=48, precision="bf16x3")
    d = FMMPlan(torch.tensor(1.01 * x, device="cuda"), kernel="laplace", p=6, ncrit=64, precision="bf16x3")
    e = FMMPlan(xt, kernel="laplace", p=6, ncrit=64, precision="bf16x3")
    assert c.info()["tree_shared"] == 0 and d.info()["tree_shared"] == 0
    assert e.info()["tree_shared"] == 1  # from b, which holds the tree alone now


@pytest.mark.parametrize("setting", [
    {"near_early": 450, "gemm_lat": 0, "gemm_narrow": 1},
    {"near_early": 500, "m2l_early": 1},
    {"pair_order": 2},
    {"pair_order": 4, "near_early": 400, "near_early_start": 1},
])
@pytest.mark.parametrize("grad", [True, False])
def test_pair_monopole_dipole_under_other_tunables_equals_the_defaults(setting, grad):
    """The monopole + dipole pair evaluation (the direct formulation's step)
    under the pass-order and split tunables gives the default setting's
    results within single-precision rounding."""
    torch = require_gpu()
    from paper_2103_01048_amd import FMMPlan, autotune as at, eval_pair_md
    x = _cloud(6000, seed=141)
    rng = np.random.default_rng(141)
    q = torch.tensor(rng.standard_normal(len(x)), device="cuda", dtype=torch.float32)
    dip = torch.tensor(rng.standard_normal((len(x), 3)), device="cuda", dtype=torch.float32)
    xt = torch.tensor(x, device="cuda")

    def run():
        a = FMMPlan(xt, kernel="laplace", p=6, ncrit=48, precision="bf16x3")
        b = FMMPlan(xt, kernel="yukawa", kappa=KAPPA, p=6, ncrit=48, precision="bf16x3")
        assert a.info()["max_level"] >= 3
        out = eval_pair_md(a, b, q, dip, -1.0, -0.05, gradient=grad)
        return [t for o in out for t in (o if isinstance(o, tuple) else (o,))]

    ref = run()
    with at.tuning(**setting):
        got = run()
    for r, g in zip(ref, got):
        assert _rel(g, r) < 1e-6
