"""Kernel-independent fast multipole method, pass by pass, in FP64 NumPy
(Methods, Fast multipole method: equivalent and check surfaces, the matching
equations for the upward and downward equivalent densities, the P2M, M2M,
M2L, L2L, L2P and P2P operators, and the pass order: P2M at the leaves, M2M
in post-order, M2L, then L2L in pre-order with L2P and P2P at the leaves).

TEST INFRASTRUCTURE ONLY (see the package docstring).  Small inputs only.

Readings (the paper leaves these open):
  * Expansion order p = points per edge of a p x p x p grid on a cube; the
    surface keeps the grid points with a coordinate on a face:
    n = 6 (p-1)^2 + 2 points, ordered by (i, j, k) lexicographically.
  * Surface of box B (centre c, half-width h) at radius alpha:
    c + alpha h (2i/(p-1) - 1, 2j/(p-1) - 1, 2k/(p-1) - 1).
    Upward equivalent 1.05, upward check 2.95, downward equivalent 2.95,
    downward check 1.05.
  * The matching equations are solved with the truncated-SVD pseudo-inverse
    of the check-from-equivalent kernel matrix; singular values below
    tau * s_max are dropped.
  * Adaptive-tree lists U/V/W/X as in oracle.tree: V-list boxes go through
    M2L, W-list boxes through their upward equivalent densities (M2P),
    X-list boxes through their sources evaluated on the downward check
    surface (P2L), U-list leaves directly (P2P).
  * The default (direct_small=False) is the plain method: every W-list box
    acts through its upward equivalent density (M2P) and every X-list box
    through its sources evaluated on the downward check surface (P2L).
    With direct_small=True a W-list box holding at most n points contributes
    its points directly instead of its n equivalent points, and a leaf with
    at most n points takes its X-list sources directly at its points instead
    of through its check surface: both replace an approximation by the exact
    sum it approximates, so the two variants agree to within the expansion
    error (a pinned property); the GPU library takes the same shortcut, and
    its per-pass parity test asks for this variant explicitly.
"""
from __future__ import annotations

import math
from dataclasses import dataclass

import numpy as np

from . import tree as _tree

ALPHA_UE, ALPHA_UC, ALPHA_DE, ALPHA_DC = 1.05, 2.95, 2.95, 1.05


def surface_grid(p: int) -> np.ndarray:
    pts = []
    for i in range(p):
        for j in range(p):
            for k in range(p):
                if min(i, j, k) == 0 or max(i, j, k) == p - 1:
                    pts.append((2.0 * i / (p - 1) - 1.0, 2.0 * j / (p - 1) - 1.0,
                                2.0 * k / (p - 1) - 1.0))
    return np.array(pts, dtype=np.float64)


def kernel_matrix(X, Y, kernel, kappa):
    d = X[:, None, :] - Y[None, :, :]
    r = np.sqrt(np.sum(d * d, axis=2))
    with np.errstate(divide="ignore"):
        if kernel == "yukawa":
            g = np.exp(-kappa * r) / (4 * math.pi * r)
        else:
            g = 1.0 / (4 * math.pi * r)
    g[r == 0] = 0.0
    return g


def kernel_grad(X, Y, kernel, kappa):
    """d/dX of g(X_i, Y_j): (nx, ny, 3)."""
    d = X[:, None, :] - Y[None, :, :]
    r = np.sqrt(np.sum(d * d, axis=2))
    with np.errstate(divide="ignore", invalid="ignore"):
        if kernel == "yukawa":
            f = -(1 + kappa * r) * np.exp(-kappa * r) / (4 * math.pi * r ** 3)
        else:
            f = -1.0 / (4 * math.pi * r ** 3)
    f[r == 0] = 0.0
    return f[:, :, None] * d


def pinv_tsvd(A, tau):
    U, s, Vt = np.linalg.svd(A)
    keep = s > tau * s[0]
    sinv = np.zeros_like(s)
    sinv[keep] = 1.0 / s[keep]
    return (Vt.T * sinv) @ U.T


@dataclass
class Operators:
    uc2e: dict   # level -> (n,n)
    dc2e: dict
    m2m: dict    # (level, octant) -> (n,n)  child level+1 -> parent level
    l2l: dict    # (level, octant) -> (n,n)  parent level -> child check
    m2l: dict    # (level, (ox,oy,oz)) -> (n,n)


def precompute(t: _tree.Tree, p: int, kernel: str, kappa: float, tau: float) -> Operators:
    grid = surface_grid(p)
    levels = sorted(set(int(l) for l in t.level))
    ops = Operators({}, {}, {}, {}, {})
    for l in levels:
        h = t.W / (1 << (l + 1))
        ue, uc = ALPHA_UE * h * grid, ALPHA_UC * h * grid
        de, dc = ALPHA_DE * h * grid, ALPHA_DC * h * grid
        ops.uc2e[l] = pinv_tsvd(kernel_matrix(uc, ue, kernel, kappa), tau)
        ops.dc2e[l] = pinv_tsvd(kernel_matrix(dc, de, kernel, kappa), tau)
    for l in levels:
        if l + 1 not in ops.uc2e:
            continue
        h = t.W / (1 << (l + 1))
        hc = h / 2
        for c in range(8):
            off = np.array([(c >> 2) & 1, (c >> 1) & 1, c & 1], dtype=np.float64) * 2 - 1
            off *= hc
            ue_child = ALPHA_UE * hc * grid + off
            ops.m2m[(l, c)] = ops.uc2e[l] @ kernel_matrix(ALPHA_UC * h * grid, ue_child, kernel, kappa)
            dc_child = ALPHA_DC * hc * grid + off
            ops.l2l[(l, c)] = kernel_matrix(dc_child, ALPHA_DE * h * grid, kernel, kappa)
    return ops


def _m2l_matrix(ops, t, p, grid, l, o, kernel, kappa):
    key = (l, o)
    if key not in ops.m2l:
        h = t.W / (1 << (l + 1))
        src = ALPHA_UE * h * grid + 2 * h * np.array(o, dtype=np.float64)
        ops.m2l[key] = kernel_matrix(ALPHA_DC * h * grid, src, kernel, kappa)
    return ops.m2l[key]


@dataclass
class FMMResult:
    pot: np.ndarray
    grad: np.ndarray
    equ: np.ndarray      # upward equivalent densities per box (nbox, n)
    chk_d: np.ndarray    # downward check potentials per box
    eqd: np.ndarray      # downward equivalent densities per box


def evaluate(x, q, kernel="laplace", kappa=0.0, p=6, ncrit=64, tau=1e-14, t=None, ops=None,
             direct_small=False):
    """FMM potential and gradient at every point from densities q (targets =
    sources = x; zero-distance pairs excluded).  Returns FMMResult in the
    caller's point order."""
    x = np.asarray(x, dtype=np.float64)
    q = np.asarray(q, dtype=np.float64)
    if t is None:
        t = _tree.build_tree(x, ncrit)
    if ops is None:
        ops = precompute(t, p, kernel, kappa, tau)
    grid = surface_grid(p)
    n = len(grid)
    xs = x[t.perm]
    qs = q[t.perm]
    nb = t.nbox
    equ = np.zeros((nb, n))
    chk = np.zeros((nb, n))
    eqd = np.zeros((nb, n))
    cen = np.array([t.center(b) for b in range(nb)])
    hh = np.array([t.half(b) for b in range(nb)])
    maxl = int(t.level.max())

    # upward pass: P2M at leaves, M2M in post-order (deepest level first)
    for l in range(maxl, -1, -1):
        for b in np.nonzero(t.level == l)[0]:
            if t.is_leaf(b):
                s = slice(t.begin[b], t.end[b])
                uc = ALPHA_UC * hh[b] * grid + cen[b]
                equ[b] = ops.uc2e[l] @ (kernel_matrix(uc, xs[s], kernel, kappa) @ qs[s])
            else:
                acc = np.zeros(n)
                for ch in range(t.child_begin[b], t.child_begin[b] + t.nchild[b]):
                    acc += ops.m2m[(l, _octant(t, ch))] @ equ[ch]
                equ[b] = acc

    # interaction pass: M2L over V lists, P2L over X lists
    for b in range(nb):
        l = int(t.level[b])
        for a in t.V[b]:
            o = tuple(int(v) for v in (t.anchor[a] - t.anchor[b]))
            chk[b] += _m2l_matrix(ops, t, p, grid, l, o, kernel, kappa) @ equ[a]
        x_direct = direct_small and t.is_leaf(b) and (t.end[b] - t.begin[b]) <= n
        if t.X[b] and not x_direct:
            dc = ALPHA_DC * hh[b] * grid + cen[b]
            for a in t.X[b]:
                s = slice(t.begin[a], t.end[a])
                chk[b] += kernel_matrix(dc, xs[s], kernel, kappa) @ qs[s]

    # downward pass in pre-order (coarsest level first)
    for l in range(0, maxl + 1):
        for b in np.nonzero(t.level == l)[0]:
            eqd[b] = ops.dc2e[l] @ chk[b]
            for ch in range(t.child_begin[b], t.child_begin[b] + t.nchild[b]) if t.nchild[b] else ():
                chk[ch] += ops.l2l[(l, _octant(t, ch))] @ eqd[b]

    # leaves: L2P, M2P (W list), P2P (U list)
    pot = np.zeros(len(x))
    grad = np.zeros((len(x), 3))
    for b in range(nb):
        if not t.is_leaf(b):
            continue
        s = slice(t.begin[b], t.end[b])
        tx = xs[s]
        de = ALPHA_DE * hh[b] * grid + cen[b]
        pot[s] += kernel_matrix(tx, de, kernel, kappa) @ eqd[b]
        grad[s] += np.einsum("ijd,j->id", kernel_grad(tx, de, kernel, kappa), eqd[b])
        direct = list(t.U[b])
        for a in t.W_[b]:
            if direct_small and t.end[a] - t.begin[a] <= n:
                direct.append(a)
                continue
            ue = ALPHA_UE * hh[a] * grid + cen[a]
            pot[s] += kernel_matrix(tx, ue, kernel, kappa) @ equ[a]
            grad[s] += np.einsum("ijd,j->id", kernel_grad(tx, ue, kernel, kappa), equ[a])
        if direct_small and (t.end[b] - t.begin[b]) <= n:
            direct += list(t.X[b])
        for a in direct:
            sa = slice(t.begin[a], t.end[a])
            pot[s] += kernel_matrix(tx, xs[sa], kernel, kappa) @ qs[sa]
            grad[s] += np.einsum("ijd,j->id", kernel_grad(tx, xs[sa], kernel, kappa), qs[sa])

    out_p = np.empty_like(pot)
    out_g = np.empty_like(grad)
    out_p[t.perm] = pot
    out_g[t.perm] = grad
    return FMMResult(out_p, out_g, equ, chk, eqd)


def _octant(t, b):
    a = t.anchor[b]
    return int(((a[0] & 1) << 2) | ((a[1] & 1) << 1) | (a[2] & 1))
