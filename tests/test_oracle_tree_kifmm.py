"""Pins of the octree/list oracle (exactly-once coverage of every target-
source pair, leaf sizes, Morton order) and of the FP64 KIFMM oracle (error
of the potential and of the gradient against the direct sum falls with the
expansion order, on the plain method and on a deep adaptive tree whose W and
X lists hold boxes larger than the surfaces; the variant that takes small
W/X boxes directly agrees with the plain one to within the expansion error;
dropping a far-field stage is detected; a single leaf is the exact direct
sum)."""
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
    errs, gerrs = [], []
    for p in (3, 5, 7):
        r = kifmm.evaluate(x, q, kernel, kappa, p=p, ncrit=32, t=t, tau=1e-11)
        errs.append(D.rel_l2(r.pot, p0))
        gerrs.append(D.rel_l2(r.grad, g0))
    assert errs[0] < 2e-2 and errs[1] < 1e-4 and errs[2] < 2e-6, errs
    assert errs[0] > 5 * errs[1] > 25 * errs[2], errs
    # the gradient (L2P and M2P through the kernel's gradient) converges too
    assert gerrs[0] < 5e-2 and gerrs[1] < 5e-4 and gerrs[2] < 2e-5, gerrs
    assert gerrs[0] > 5 * gerrs[1] > 25 * gerrs[2], gerrs


def _clustered():
    """A dense cluster inside a sparse cloud: a deep tree (8 levels at ncrit
    24) whose W and X lists are long and hold boxes of more than the 56
    surface points of p = 4, so both the surface (M2P, P2L) and the direct
    forms of those lists are exercised."""
    rng = np.random.default_rng(21)
    x = np.concatenate([rng.normal(0, 0.02, (800, 3)), rng.uniform(-1, 1, (1200, 3))])
    return x, rng.standard_normal(len(x))


@pytest.mark.parametrize("kernel,kappa", [("laplace", 0.0), ("yukawa", 2.0)])
def test_plain_method_on_adaptive_tree(kernel, kappa):
    """The plain method (every W box through M2P from its upward equivalent
    surface, every X box through P2L on the downward check surface) on a
    tree with 2,278 W and X entries: potential and gradient errors fall with
    p; the shortcut variant agrees with it to within the expansion error."""
    x, q = _clustered()
    t = T.build_tree(x, 24)
    nw = sum(len(v) for v in t.W_)
    assert int(t.level.max()) >= 7 and nw > 2000 and nw == sum(len(v) for v in t.X)
    p0, g0 = D.direct(x, x, q, kernel, kappa)
    errs, gerrs = [], []
    for p in (3, 5):
        r = kifmm.evaluate(x, q, kernel, kappa, p=p, ncrit=24, t=t, tau=1e-11)
        errs.append(D.rel_l2(r.pot, p0))
        gerrs.append(D.rel_l2(r.grad, g0))
    # measured: pot 3.1e-3, 3.8e-5; grad 3.1e-3, 7.9e-5 (both kernels)
    assert errs[0] < 1e-2 and errs[1] < 1e-4 and errs[0] > 20 * errs[1], errs
    assert gerrs[0] < 1e-2 and gerrs[1] < 2e-4 and gerrs[0] > 10 * gerrs[1], gerrs
    rs = kifmm.evaluate(x, q, kernel, kappa, p=5, ncrit=24, t=t, tau=1e-11, direct_small=True)
    es, gs = D.rel_l2(rs.pot, p0), D.rel_l2(rs.grad, g0)
    assert es < 1e-4 and gs < 2e-4
    # the two variants differ by less than either one's expansion error
    assert D.rel_l2(r.pot, rs.pot) < max(errs[1], es)
    assert D.rel_l2(r.grad, rs.grad) < max(gerrs[1], gs)


@pytest.mark.parametrize("drop", ["W", "X", "WX"])
def test_dropping_w_or_x_is_detected(drop):
    """Dropping the M2P (W) or the P2L (X) contributions of the plain method
    leaves an error far outside what the expansion order allows."""
    x, q = _clustered()
    t = T.build_tree(x, 24)
    p0, g0 = D.direct(x, x, q)
    saved = t.W_, t.X
    if "W" in drop:
        t.W_ = [[] for _ in saved[0]]
    if "X" in drop:
        t.X = [[] for _ in saved[1]]
    r = kifmm.evaluate(x, q, p=4, ncrit=24, t=t, tau=1e-11)
    t.W_, t.X = saved
    assert max(D.rel_l2(r.pot, p0), D.rel_l2(r.grad, g0)) > 1e-2


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
