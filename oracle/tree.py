"""Adaptive octree and interaction lists of the fast multipole method
(Methods, Fast multipole method: enclosing cube, recursive subdivision until a
leaf holds at most a constant number of points, near field N(B) and
interaction list I(B)), written plainly in Python for small inputs.

TEST INFRASTRUCTURE ONLY (see the package docstring).

Readings (the paper gives only the uniform-tree picture):
  * Root cube: centre = midpoint of the bounding box, side
    W = (largest extent) * (1 + 2^-20) (W = 1 for a zero extent),
    lower corner lo = centre - W/2.
  * Morton key: cell_d = floor(((x_d - lo_d) / W) * 2^21) clamped to
    [0, 2^21 - 1]; bits interleaved x,y,z from the most significant level,
    child octant = 4*xbit + 2*ybit + zbit.  Points are stably sorted by key.
  * A box splits while it holds more than ncrit points and its level is
    below 21; empty children are not created.
  * Boxes are numbered by (level, key) ascending: root 0, each level in
    Morton order.
  * Lists for an adaptive tree (the near field split into U and W, X, the
    interaction list called V):
      U(B), leaf B:   leaves adjacent to B (B included)
      V(B):           children of the parent's same-level neighbours that are
                      not adjacent to B (the paper's I(B))
      W(B), leaf B:   descendants of B's same-level neighbours that are not
                      adjacent to B but whose parent is
      X(B):           boxes A with B in W(A)
    Two boxes are adjacent when their closed cubes intersect.
"""
from __future__ import annotations

from dataclasses import dataclass, field

import numpy as np

MAXLEVEL = 21


def root_cube(x: np.ndarray):
    mn = x.min(axis=0)
    mx = x.max(axis=0)
    center = (mn + mx) * 0.5
    ext = float(np.max(mx - mn))
    W = ext * (1.0 + 2.0 ** -20) if ext > 0 else 1.0
    lo = center - 0.5 * W
    return lo, W


def morton_cells(x: np.ndarray, lo: np.ndarray, W: float) -> np.ndarray:
    t = (x - lo[None, :]) / W
    c = np.floor(t * 2097152.0)
    return np.clip(c, 0, 2 ** 21 - 1).astype(np.int64)


def interleave(cells: np.ndarray) -> np.ndarray:
    key = np.zeros(len(cells), dtype=np.int64)
    for b in range(21):
        for d in range(3):
            bit = (cells[:, d] >> b) & 1
            key |= bit << (3 * b + (2 - d))
    return key


@dataclass
class Tree:
    lo: np.ndarray
    W: float
    keys: np.ndarray        # sorted keys (N,)
    perm: np.ndarray        # sorted position -> original index
    level: np.ndarray       # per box
    anchor: np.ndarray      # (nbox, 3) integer coordinates at the box level
    begin: np.ndarray
    end: np.ndarray
    parent: np.ndarray
    child_begin: np.ndarray
    nchild: np.ndarray
    U: list = field(default_factory=list)
    V: list = field(default_factory=list)
    W_: list = field(default_factory=list)
    X: list = field(default_factory=list)

    @property
    def nbox(self):
        return len(self.level)

    def is_leaf(self, b):
        return self.nchild[b] == 0

    def center(self, b):
        l = self.level[b]
        s = self.W / (1 << l)
        return self.lo + (self.anchor[b] + 0.5) * s

    def half(self, b):
        return self.W / (1 << (self.level[b] + 1))


def _adjacent(la, aa, lb, ab) -> bool:
    sa = 1 << (MAXLEVEL - la)
    sb = 1 << (MAXLEVEL - lb)
    for d in range(3):
        loa, lob = aa[d] * sa, ab[d] * sb
        if loa > lob + sb or lob > loa + sa:
            return False
    return True


def build_tree(x: np.ndarray, ncrit: int) -> Tree:
    x = np.asarray(x, dtype=np.float64)
    n = len(x)
    lo, W = root_cube(x)
    cells = morton_cells(x, lo, W)
    keys = interleave(cells)
    perm = np.argsort(keys, kind="stable")
    skeys = keys[perm]

    # boxes as (level, prefix, begin, end); breadth first, Morton order per level
    boxes = [(0, 0, 0, n)]
    parent = [-1]
    levels = [[0]]
    while True:
        nxt = []
        for b in levels[-1]:
            l, pre, bg, en = boxes[b]
            if en - bg <= ncrit or l >= MAXLEVEL:
                continue
            shift = 3 * (MAXLEVEL - (l + 1))
            digits = (skeys[bg:en] >> shift) & 7
            for c in range(8):
                idx = np.nonzero(digits == c)[0]
                if len(idx) == 0:
                    continue
                cb, ce = bg + idx[0], bg + idx[-1] + 1
                boxes.append((l + 1, (pre << 3) | c, cb, ce))
                parent.append(b)
                nxt.append(len(boxes) - 1)
        if not nxt:
            break
        levels.append(nxt)
    nb = len(boxes)
    level = np.array([b[0] for b in boxes], dtype=np.int32)
    prefix = np.array([b[1] for b in boxes], dtype=np.int64)
    begin = np.array([b[2] for b in boxes], dtype=np.int64)
    end = np.array([b[3] for b in boxes], dtype=np.int64)
    parent = np.array(parent, dtype=np.int64)
    anchor = np.zeros((nb, 3), dtype=np.int64)
    for b in range(nb):
        pre, l = int(prefix[b]), int(level[b])
        a = [0, 0, 0]
        for k in range(l):
            dig = (pre >> (3 * (l - 1 - k))) & 7
            a[0] = (a[0] << 1) | ((dig >> 2) & 1)
            a[1] = (a[1] << 1) | ((dig >> 1) & 1)
            a[2] = (a[2] << 1) | (dig & 1)
        anchor[b] = a
    child_begin = -np.ones(nb, dtype=np.int64)
    nchild = np.zeros(nb, dtype=np.int32)
    for b in range(1, nb):
        p = parent[b]
        if child_begin[p] < 0:
            child_begin[p] = b
        nchild[p] += 1
    t = Tree(lo, W, skeys, perm, level, anchor, begin, end, parent, child_begin, nchild)
    _build_lists(t)
    return t


def _build_lists(t: Tree):
    nb = t.nbox
    lookup = {}
    for b in range(nb):
        lookup[(int(t.level[b]),) + tuple(int(v) for v in t.anchor[b])] = b

    def find(l, a):
        return lookup.get((l, a[0], a[1], a[2]))

    def adj(a, b):
        return _adjacent(int(t.level[a]), t.anchor[a], int(t.level[b]), t.anchor[b])

    def children(b):
        return range(t.child_begin[b], t.child_begin[b] + t.nchild[b]) if t.nchild[b] else range(0)

    def colleagues(b):
        l = int(t.level[b])
        a = t.anchor[b]
        out = []
        for dx in (-1, 0, 1):
            for dy in (-1, 0, 1):
                for dz in (-1, 0, 1):
                    if dx == dy == dz == 0:
                        continue
                    c = find(l, (a[0] + dx, a[1] + dy, a[2] + dz))
                    if c is not None:
                        out.append(c)
        return out

    U = [[] for _ in range(nb)]
    V = [[] for _ in range(nb)]
    Wl = [[] for _ in range(nb)]
    X = [[] for _ in range(nb)]
    for b in range(nb):
        # V list
        if t.level[b] >= 2:
            p = t.parent[b]
            for c in [p] + colleagues(p):
                for ch in children(c):
                    if not adj(ch, b):
                        V[b].append(ch)
        if not t.is_leaf(b):
            continue
        # U and W lists of leaf b
        l = int(t.level[b])
        a = t.anchor[b]
        uset = set()
        for dx in (-1, 0, 1):
            for dy in (-1, 0, 1):
                for dz in (-1, 0, 1):
                    cell = (a[0] + dx, a[1] + dy, a[2] + dz)
                    if min(cell) < 0 or max(cell) >= (1 << l):
                        continue
                    ll = l
                    box = None
                    cc = cell
                    while ll >= 0:
                        box = find(ll, cc)
                        if box is not None:
                            break
                        ll -= 1
                        cc = (cc[0] >> 1, cc[1] >> 1, cc[2] >> 1)
                    if box is None:
                        continue
                    if t.is_leaf(box):
                        uset.add(box)
                    elif ll == l:
                        stack = list(children(box))
                        while stack:
                            d = stack.pop()
                            if adj(d, b):
                                if t.is_leaf(d):
                                    uset.add(d)
                                else:
                                    stack.extend(children(d))
                            else:
                                Wl[b].append(d)
        U[b] = sorted(uset)
        Wl[b] = sorted(set(Wl[b]))
    for b in range(nb):
        for a in Wl[b]:
            X[a].append(b)
    t.U = [sorted(u) for u in U]
    t.V = [sorted(v) for v in V]
    t.W_ = [sorted(w) for w in Wl]
    t.X = [sorted(x) for x in X]


def csr(lists):
    off = np.zeros(len(lists) + 1, dtype=np.int64)
    for i, l in enumerate(lists):
        off[i + 1] = off[i] + len(l)
    idx = np.array([v for l in lists for v in l], dtype=np.int64)
    return off, idx
