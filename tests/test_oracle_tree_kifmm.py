"""Pins of the octree/list oracle (exactly-once coverage of every target-
source pair, leaf sizes, Morton order) and of the FP64 KIFMM oracle (error
against the direct sum falls with the expansion order; a single leaf is the
exact direct sum)."""
import numpy as np
import pytest

import synth
from oracle import direct as D
from oracle import kifmm, tree as T


def _clouds():
    rng = np.random.default_rng(11)
    yield rng.uniform(0, 1, (300, 3)), 8
    x, _ = synth.unit_sphere_cloud(500, seed=12)
    yield x, 10
    # clustered cloud: deep, very adaptive tree
    c = np.concatenate([rng.normal(0, 0.01, (150, 3)), rng.uniform(-1, 1, (150, 3))])
    yield c, 6
    # duplicated points beyond ncrit stop at the level cap
    yield np.concatenate([np.zeros((12, 3)), rng.uniform(0, 1, (40, 3))]), 4


def _ancestors(t, b):
    out = [b]
    while t.parent[b] >= 0:
        b = t.parent[b]
        out.append(b)
    return out


@pytest.mark.parametrize("case", range(4))
def test_every_pair_covered_exactly_once(case):
    x, ncrit = list(_clouds())[case]
    t = T.build_tree(x, ncrit)
    leaves = [b for b in range(t.nbox) if t.is_leaf(b)]
    for B in leaves:
        anc_b = _ancestors(t, B)
        for A in leaves:
            anc_a = set(_ancestors(t, A))
            cnt = 0
            cnt += A in t.U[B]
            cnt += sum(1 for bb in anc_b for v in t.V[bb] if v in anc_a)
            cnt += sum(1 for w in t.W_[B] if w in anc_a)
            cnt += sum(1 for bb in anc_b for xx in t.X[bb] if xx == A)
            assert cnt == 1, (B, A, cnt)


@pytest.mark.parametrize("case", range(4))
def test_tree_structure(case):
    x, ncrit = list(_clouds())[case]
    t = T.build_tree(x, ncrit)
    assert np.all(np.diff(t.keys) >= 0)
    assert sorted(t.perm.tolist()) == list(range(len(x)))
    seen = np.zeros(len(x), dtype=int)
    for b in range(t.nbox):
        if t.is_leaf(b):
            seen[t.begin[b]:t.end[b]] += 1
            assert t.end[b] - t.begin[b] <= ncrit or t.level[b] == T.MAXLEVEL
        else:
            ch = range(t.child_begin[b], t.child_begin[b] + t.nchild[b])
            assert t.begin[ch[0]] == t.begin[b] and t.end[ch[-1]] == t.end[b]
        # every point of the box lies inside its (closed) cube
        c, h = t.center(b), t.half(b)
        pts = x[t.perm[t.begin[b]:t.end[b]]]
        assert np.all(np.abs(pts - c) <= h * (1 + 1e-12))
    assert np.all(seen == 1)
    # numbering by (level, key)
    lv = t.level
    assert np.all(np.diff(lv) >= 0)


def test_stable_order_of_equal_keys():
    x = np.array([[0.1, 0.1, 0.1]] * 5 + [[0.9, 0.9, 0.9]] * 3)
    t = T.build_tree(x, 2)
    assert t.perm[:5].tolist() == [0, 1, 2, 3, 4]


@pytest.mark.parametrize("kernel", ["laplace", "yukawa"])
def test_single_leaf_is_direct_sum(kernel):
    x, q = synth.unit_sphere_cloud(200, seed=13)
    r = kifmm.evaluate(x, q, kernel, 0.125, p=4, ncrit=256)
    p0, g0 = D.direct(x, x, q, kernel, 0.125)
    np.testing.assert_allclose(r.pot, p0, rtol=1e-12, atol=1e-14)
    np.testing.assert_allclose(r.grad, g0, rtol=1e-12, atol=1e-13)


@pytest.mark.parametrize("kernel,kappa", [("laplace", 0.0), ("yukawa", 2.0)])
def test_error_falls_with_order(kernel, kappa):
    x, q = synth.unit_sphere_cloud(3000, seed=14)
    p0, g0 = D.direct(x, x, q, kernel, kappa)
    t = T.build_tree(x, 32)
    assert int(t.level.max()) >= 3 and sum(len(v) for v in t.V) > 1000
    errs = []
    for p in (3, 5, 7):
        r = kifmm.evaluate(x, q, kernel, kappa, p=p, ncrit=32, t=t, tau=1e-11)
        errs.append(D.rel_l2(r.pot, p0))
    assert errs[0] < 2e-2 and errs[1] < 1e-4 and errs[2] < 2e-6, errs
    assert errs[0] > 5 * errs[1] > 25 * errs[2], errs


def test_dropping_m2l_is_detected():
    """A plausible mistake (a whole far-field stage missing) is far outside
    the tolerance the error-vs-order pin allows."""
    x, q = synth.unit_sphere_cloud(2000, seed=15)
    p0, _ = D.direct(x, x, q)
    t = T.build_tree(x, 32)
    saved = t.V
    t.V = [[] for _ in saved]
    r = kifmm.evaluate(x, q, p=5, ncrit=32, t=t)
    t.V = saved
    assert D.rel_l2(r.pot, p0) > 1e-2
