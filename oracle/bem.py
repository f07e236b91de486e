"""Dense P0 Galerkin boundary-element oracle for the direct formulation of
the linearised Poisson-Boltzmann interface problem (Methods: the integral
representation, the single- and double-layer operators, the direct
formulation, the reaction potential and the polar solvation energy; the
split of the discrete operator into a regular quadrature-point sum plus a
singular correction, FMM-accelerated evaluation of integral operators).

TEST INFRASTRUCTURE ONLY (see the package docstring).  FP64, dense, small
meshes.

Discretisation (readings where the paper is silent):
  * Triangles with counter-clockwise vertices seen from the solvent; unit
    normal n_t = (v1 - v0) x (v2 - v0) / |.| points out of the molecule.
  * P0 trial and test functions; unknowns u_t (potential) and v_t (its
    normal derivative from the solute side) per triangle.
  * Regular quadrature: 3-point rule (barycentric (2/3, 1/6, 1/6) and
    permutations, weights 1/3) or the 6-point degree-4 rule.
  * Operator entries for a pair (s, t):
      V[s,t] = int_Ts int_Tt g(x, y),  K[s,t] = int_Ts int_Tt dg/dn_y(x, y)
    with dg/dn_y = n_t . (x - y) (1 + kappa r) exp(-kappa r) / (4 pi r^3).
    Pairs that share no vertex use the regular rule on both triangles (the
    same sums the quadrature-point FMM evaluates).  Pairs that share a vertex
    (identical, edge- or vertex-adjacent) use the singular rule below; the
    difference between the two rules is the correction S - C of the split
    A = P2^T (G - C) P1 + S.
  * Singular rule: the Laplace part of the inner integral over the flat
    trial triangle in closed form -- the potential of a uniform triangle
    (sum over edges of logarithm and arctangent terms) and, for the double
    layer, minus the signed solid angle of the triangle (Van Oosterom and
    Strackee's formula) -- integrated over the test triangle with an n x n
    collapsed Gauss-Legendre rule; the Yukawa remainder
    (exp(-kappa r) - 1) / (4 pi r) and its normal derivative are bounded and
    use an m x m collapsed rule on both triangles.
  * System (2T unknowns):
      [ M/2 + K_L    -V_L           ] [u]   [b]
      [ M/2 - K_Y    (eps1/eps2) V_Y] [v] = [0],   M = diag(area)
    b_s = int_Ts (1/eps1) sum_k q_k g_L(x, r_k).
  * Reaction potential at the charges: sum over quadrature points of
    W_j [-dg_L/dn_y(r_k, y_j) u_t + g_L(r_k, y_j) v_t]; energy
    dG = 1/2 sum_k q_k phi_reac(r_k) * 4 pi * 332.0637 kcal/mol (the 4 pi
    undoes the 1/(4 pi) of g).
"""
from __future__ import annotations

import math
from dataclasses import dataclass

import numpy as np

from .analytic import KCAL_PER_MOL

FOUR_PI = 4.0 * math.pi


# ---------------------------------------------------------------------------
# quadrature rules on the reference triangle (barycentric coordinates)
# ---------------------------------------------------------------------------
def regular_rule(npts: int):
    """(bary (k,3), weights (k,)) with sum of weights 1."""
    if npts == 1:
        return np.array([[1 / 3, 1 / 3, 1 / 3]]), np.array([1.0])
    if npts == 3:
        b = np.array([[2 / 3, 1 / 6, 1 / 6], [1 / 6, 2 / 3, 1 / 6], [1 / 6, 1 / 6, 2 / 3]])
        return b, np.full(3, 1 / 3)
    if npts == 6:
        a1, w1 = 0.445948490915965, 0.223381589678011
        a2, w2 = 0.091576213509771, 0.109951743655322
        b = np.array([[a1, a1, 1 - 2 * a1], [a1, 1 - 2 * a1, a1], [1 - 2 * a1, a1, a1],
                      [a2, a2, 1 - 2 * a2], [a2, 1 - 2 * a2, a2], [1 - 2 * a2, a2, a2]])
        return b, np.array([w1, w1, w1, w2, w2, w2])
    raise ValueError("regular rule with 1, 3 or 6 points")


def collapsed_rule(n: int):
    """n*n collapsed Gauss-Legendre rule: point v0 + xi (v1 - v0) + xi eta
    (v2 - v1) for Gauss nodes xi, eta on [0,1]; weights (sum 1) include the
    Jacobian 2 xi."""
    g, w = np.polynomial.legendre.leggauss(n)
    g = 0.5 * (g + 1)
    w = 0.5 * w
    bary, wt = [], []
    for i in range(n):
        for j in range(n):
            xi, eta = g[i], g[j]
            l1 = xi * (1 - eta)
            l2 = xi * eta
            bary.append([1 - xi, l1, l2])
            wt.append(2 * xi * w[i] * w[j])
    return np.array(bary), np.array(wt)


# ---------------------------------------------------------------------------
# closed-form inner integrals over a flat triangle (Laplace, without 1/4pi)
# ---------------------------------------------------------------------------
def tri_potential(x, tri, n):
    """int_T 1/|x - y| dy (the potential of a uniform unit density on the
    flat triangle T).  Batched: x (..., k, 3), tri (..., 3, 3), n (..., 3)."""
    x = np.asarray(x, dtype=np.float64)
    tri = np.asarray(tri, dtype=np.float64)
    n = np.asarray(n, dtype=np.float64)
    nn = n[..., None, :]
    d = np.sum((x - tri[..., 0:1, :]) * nn, axis=-1)
    rho = x - d[..., None] * nn
    ad = np.abs(d)
    out = np.zeros(x.shape[:-1])
    for i in range(3):
        a = tri[..., i:i + 1, :]
        b = tri[..., (i + 1) % 3:(i + 1) % 3 + 1, :]
        L = np.linalg.norm(b - a, axis=-1)
        lh = (b - a) / L[..., None]
        uh = np.cross(lh, nn)
        t0 = np.sum((a - rho) * uh, axis=-1)
        lp = np.sum((b - rho) * lh, axis=-1)
        lm = np.sum((a - rho) * lh, axis=-1)
        Rp = np.linalg.norm(x - b, axis=-1)
        Rm = np.linalg.norm(x - a, axis=-1)
        R02 = t0 * t0 + d * d
        with np.errstate(divide="ignore", invalid="ignore"):
            lg = np.log((Rp + lp) / (Rm + lm))
        lg = np.where(np.abs(t0) > 1e-14 * L, lg, 0.0)
        out += t0 * lg
        out -= ad * (np.arctan2(t0 * lp, R02 + ad * Rp) - np.arctan2(t0 * lm, R02 + ad * Rm))
    return out


def tri_dlp(x, tri, n):
    """int_T n . (x - y) / |x - y|^3 dy: minus the signed solid angle of T
    seen from x (Van Oosterom-Strackee); for x in the plane of T the value
    is the principal value 0.  Batched like tri_potential."""
    x = np.asarray(x, dtype=np.float64)
    tri = np.asarray(tri, dtype=np.float64)
    R1, R2, R3 = tri[..., 0:1, :] - x, tri[..., 1:2, :] - x, tri[..., 2:3, :] - x
    r1, r2, r3 = (np.linalg.norm(R, axis=-1) for R in (R1, R2, R3))
    num = np.sum(R1 * np.cross(R2, R3), axis=-1)
    den = (r1 * r2 * r3 + np.sum(R1 * R2, axis=-1) * r3 + np.sum(R1 * R3, axis=-1) * r2
           + np.sum(R2 * R3, axis=-1) * r1)
    om = -2.0 * np.arctan2(num, den)
    return np.where(np.abs(num) <= 1e-13 * r1 * r2 * r3, 0.0, om)


# ---------------------------------------------------------------------------
# mesh data
# ---------------------------------------------------------------------------
@dataclass
class Mesh:
    verts: np.ndarray
    tris: np.ndarray
    area: np.ndarray
    normal: np.ndarray
    qpts: np.ndarray     # (T, k, 3)
    qw: np.ndarray       # (T, k) = rule weight * area


def make_mesh(verts, tris, npts: int = 3) -> Mesh:
    v = np.asarray(verts, dtype=np.float64)
    t = np.asarray(tris, dtype=np.int64)
    a, b, c = v[t[:, 0]], v[t[:, 1]], v[t[:, 2]]
    cr = np.cross(b - a, c - a)
    nrm = np.linalg.norm(cr, axis=1)
    area = 0.5 * nrm
    normal = cr / nrm[:, None]
    bary, w = regular_rule(npts)
    qp = np.einsum("kj,tjd->tkd", bary, np.stack([a, b, c], axis=1))
    return Mesh(v, t, area, normal, qp, area[:, None] * w[None, :])


def singular_pairs(m: Mesh):
    """(s, t) pairs that share at least one vertex, s-major, t ascending."""
    vt = [[] for _ in range(len(m.verts))]
    for ti, tri in enumerate(m.tris):
        for vi in tri:
            vt[vi].append(ti)
    out = []
    for s, tri in enumerate(m.tris):
        nb = sorted(set(t for vi in tri for t in vt[vi]))
        out += [(s, t) for t in nb]
    return out


def _gk(r, kappa):
    return np.exp(-kappa * r) / (FOUR_PI * r)


def regular_entries(m: Mesh, s, t, kappa):
    """Regular-rule (quadrature-point) values of V and K for pair (s, t),
    zero-distance point pairs left out."""
    x = m.qpts[s]
    y = m.qpts[t]
    d = x[:, None, :] - y[None, :, :]
    r = np.linalg.norm(d, axis=2)
    ww = m.qw[s][:, None] * m.qw[t][None, :]
    mask = r > 0
    rr = np.where(mask, r, 1.0)
    g = np.where(mask, np.exp(-kappa * rr) / (FOUR_PI * rr), 0.0)
    dn = d @ m.normal[t]
    kk = np.where(mask, dn * (1 + kappa * rr) * np.exp(-kappa * rr) / (FOUR_PI * rr ** 3), 0.0)
    return float(np.sum(ww * g)), float(np.sum(ww * kk))


def singular_entries(m: Mesh, s, t, kappa, n_outer: int = 8, n_rem: int = 4):
    """Accurate V and K for pairs sharing a vertex (see the module notes).
    s, t: arrays of triangle indices (one entry per pair)."""
    s = np.atleast_1d(np.asarray(s))
    t = np.atleast_1d(np.asarray(t))
    tri_s = m.verts[m.tris[s]]            # (P,3,3)
    tri_t = m.verts[m.tris[t]]
    nt = m.normal[t]                      # (P,3)
    bo, wo = collapsed_rule(n_outer)
    xo = np.einsum("kj,pjd->pkd", bo, tri_s)
    W = wo[None, :] * m.area[s][:, None]
    V = np.sum(W * tri_potential(xo, tri_t, nt), axis=1) / FOUR_PI
    K = np.sum(W * tri_dlp(xo, tri_t, nt), axis=1) / FOUR_PI
    # on its own flat element n . (x - y) = 0: the self double layer vanishes
    # (evaluating the solid angle there only sees rounding in the plane test)
    K = np.where(s == t, 0.0, K)
    if kappa > 0:
        br, wr = collapsed_rule(n_rem)
        xr = np.einsum("kj,pjd->pkd", br, tri_s)
        yr = np.einsum("kj,pjd->pkd", br, tri_t)
        d = xr[:, :, None, :] - yr[:, None, :, :]
        r = np.linalg.norm(d, axis=-1)
        ww = (wr[None, :] * m.area[s][:, None])[:, :, None] * (wr[None, :] * m.area[t][:, None])[:, None, :]
        kr = kappa * r
        dn = np.einsum("pabd,pd->pab", d, nt)
        with np.errstate(divide="ignore", invalid="ignore"):
            remV = np.where(r > 0, np.expm1(-kr) / (FOUR_PI * r), -kappa / FOUR_PI)
            fac = (1 + kr) * np.exp(-kr) - 1.0
            remK = np.where(r > 0, dn * fac / (FOUR_PI * r ** 3), 0.0)
        V = V + np.sum(ww * remV, axis=(1, 2))
        K = K + np.where(s == t, 0.0, np.sum(ww * remK, axis=(1, 2)))
    return V, K


def operators(m: Mesh, kappa: float, n_outer: int = 8, n_rem: int = 4, chunk: int = 64):
    """Dense V and K (T x T) for one kernel (rows assembled in chunks)."""
    T = len(m.tris)
    k = m.qpts.shape[1]
    X = m.qpts.reshape(-1, 3)
    Wf = m.qw.reshape(-1)
    nY = np.repeat(m.normal, k, axis=0)
    Vq = np.zeros((T, T))
    Kq = np.zeros((T, T))
    for s0 in range(0, T, chunk):
        s1 = min(T, s0 + chunk)
        Xs = X[s0 * k:s1 * k]
        d = Xs[:, None, :] - X[None, :, :]
        r = np.sqrt(np.einsum("ijd,ijd->ij", d, d))
        mask = r > 0
        rr = np.where(mask, r, 1.0)
        e = np.exp(-kappa * rr) if kappa > 0 else 1.0
        g = np.where(mask, e / (FOUR_PI * rr), 0.0)
        dn = np.einsum("ijd,jd->ij", d, nY)
        kk = np.where(mask, dn * (1 + kappa * rr) * e / (FOUR_PI * rr ** 3), 0.0)
        ws = Wf[s0 * k:s1 * k]
        Vq[s0:s1] = (ws[:, None] * g * Wf[None, :]).reshape(s1 - s0, k, T, k).sum(axis=(1, 3))
        Kq[s0:s1] = (ws[:, None] * kk * Wf[None, :]).reshape(s1 - s0, k, T, k).sum(axis=(1, 3))
    sp = np.array(singular_pairs(m))
    Vs, Ks = singular_entries(m, sp[:, 0], sp[:, 1], kappa, n_outer, n_rem)
    Vq[sp[:, 0], sp[:, 1]] = Vs
    Kq[sp[:, 0], sp[:, 1]] = Ks
    return Vq, Kq


def system(m: Mesh, eps1: float, eps2: float, kappa: float, **kw):
    VL, KL = operators(m, 0.0, **kw)
    VY, KY = operators(m, kappa, **kw)
    M = np.diag(m.area)
    A = np.block([[0.5 * M + KL, -VL], [0.5 * M - KY, (eps1 / eps2) * VY]])
    return A


def rhs(m: Mesh, qxyz, q, eps1: float):
    X = m.qpts.reshape(-1, 3)
    d = np.linalg.norm(X[:, None, :] - np.asarray(qxyz)[None, :, :], axis=2)
    f = (np.asarray(q)[None, :] / (FOUR_PI * eps1 * d)).sum(axis=1)
    T, k = m.qw.shape
    b = (m.qw.reshape(-1) * f).reshape(T, k).sum(axis=1)
    return np.concatenate([b, np.zeros(T)])


def reaction_potential(m: Mesh, x, qxyz):
    T = len(m.tris)
    u, v = x[:T], x[T:]
    k = m.qpts.shape[1]
    Y = m.qpts.reshape(-1, 3)
    W = m.qw.reshape(-1)
    nY = np.repeat(m.normal, k, axis=0)
    uu = np.repeat(u, k) * W
    vv = np.repeat(v, k) * W
    R = np.asarray(qxyz)[:, None, :] - Y[None, :, :]
    r = np.linalg.norm(R, axis=2)
    g = 1.0 / (FOUR_PI * r)
    dgdn = np.einsum("kjd,jd->kj", R, nY) / (FOUR_PI * r ** 3)
    return -dgdn @ uu + g @ vv


def energy(m: Mesh, x, qxyz, q):
    phi = reaction_potential(m, x, qxyz)
    return 0.5 * float(np.dot(q, phi)) * FOUR_PI * KCAL_PER_MOL


def solve(m: Mesh, qxyz, q, eps1=4.0, eps2=80.0, kappa=0.125, **kw):
    A = system(m, eps1, eps2, kappa, **kw)
    b = rhs(m, qxyz, q, eps1)
    x = np.linalg.solve(A, b)
    return x, A, b


def matvec_rows(m: Mesh, rows, x, eps1=4.0, eps2=80.0, kappa=0.125, n_outer: int = 8, n_rem: int = 4):
    """Rows `rows` of A x for any mesh size, each entry a plain sum over all
    trial triangles (regular rule) with the pairs that share a vertex taken
    by the singular rule: O(N) per row through the C direct sum."""
    from . import direct as Dd
    T = len(m.tris)
    k = m.qpts.shape[1]
    rows = np.asarray(rows)
    u, v = x[:T], x[T:]
    Y = m.qpts.reshape(-1, 3)
    W = m.qw.reshape(-1)
    n_rep = np.repeat(m.normal, k, axis=0)
    uu = np.repeat(u, k) * W
    vv = np.repeat(v, k) * W
    tgt = m.qpts[rows].reshape(-1, 3)
    wt = m.qw[rows].reshape(-1)
    out = np.zeros((len(rows), 2))
    # trial triangles sharing a vertex with each test triangle, ascending
    by_row = {int(s_): np.nonzero(np.isin(m.tris, m.tris[s_]).any(axis=1))[0]
              for s_ in rows}
    for ki, (kern, kap) in enumerate((("laplace", 0.0), ("yukawa", kappa))):
        Kx = np.zeros(len(tgt))
        for d in range(3):
            _, g = Dd.direct(tgt, Y, uu * n_rep[:, d], kern, kap)
            Kx -= g[:, d]
        Vx, _ = Dd.direct(tgt, Y, vv, kern, kap)
        Kr = (wt * Kx).reshape(len(rows), k).sum(axis=1)
        Vr = (wt * Vx).reshape(len(rows), k).sum(axis=1)
        for i, s_ in enumerate(rows):
            ts = by_row[int(s_)]
            Vs, Ks = singular_entries(m, np.full(len(ts), s_), ts, kap, n_outer, n_rem)
            for j, t_ in enumerate(ts):
                Vreg, Kreg = regular_entries(m, s_, t_, kap)
                Vr[i] += (Vs[j] - Vreg) * v[t_]
                Kr[i] += (Ks[j] - Kreg) * u[t_]
        half = 0.5 * m.area[rows] * u[rows]
        if ki == 0:
            out[:, 0] = half + Kr - Vr
        else:
            out[:, 1] = half - Kr + (eps1 / eps2) * Vr
    return out


def reaction_potential_direct(m: Mesh, x, qxyz):
    """reaction_potential through the C direct sum, for meshes too large for
    the dense kernel matrix: the double-layer term sum_j (r - y_j).n_j u_j w_j
    / (4 pi |r - y_j|^3) is minus the target gradient of the single-layer sum
    with densities n_j,d u_j w_j, summed over d."""
    from . import direct as Dd
    T = len(m.tris)
    u, v = x[:T], x[T:]
    k = m.qpts.shape[1]
    Y = m.qpts.reshape(-1, 3)
    W = m.qw.reshape(-1)
    nY = np.repeat(m.normal, k, axis=0)
    uu = np.repeat(u, k) * W
    vv = np.repeat(v, k) * W
    tgt = np.ascontiguousarray(qxyz, dtype=np.float64).reshape(-1, 3)
    phi, _ = Dd.direct(tgt, Y, vv)
    for d in range(3):
        _, g = Dd.direct(tgt, Y, uu * nY[:, d])
        phi += g[:, d]
    return phi


def energy_direct(m: Mesh, x, qxyz, q):
    phi = reaction_potential_direct(m, x, qxyz)
    return 0.5 * float(np.dot(q, phi)) * FOUR_PI * KCAL_PER_MOL


# ---------------------------------------------------------------------------
# Derivative (Juffer) formulation, P0 Galerkin (Methods, eq:juffer and
# eq:adj_hyp): unknowns u = phi_1 and v = d phi_1 / dn per triangle,
#   [ (1 + e21)/2 M - (e21 K_Y - K_L)   V_Y - V_L                 ] [u]   [b1]
#   [ W_Y - W_L                         (1 + e12)/2 M + e12 K'_Y - K'_L ] [v] = [b2]
# e21 = eps2/eps1, e12 = eps1/eps2, b2_s = int_Ts dn_x of the charges'
# Coulomb potential / eps1.  With P0 Galerkin and the same rule on both
# triangles, K' is the transpose of K.  Only the difference W_Y - W_L of the
# hypersingular operators appears; its kernel is weakly singular.
# The exterior variant (eq:lu) is the same pair of equations scaled by
# eps1/eps2 and solved for the solvent-side unknowns phi_2 and d phi_2/dn;
# the interface conditions map its solution back to (u, v).
# ---------------------------------------------------------------------------
def _h_derivs(r, kappa):
    """h = (exp(-kappa r) - 1)/(4 pi r) (the Yukawa minus the Laplace
    kernel): returns h'(r), and A = h'/r - kappa^2/(8 pi r) (bounded) and
    B = h'' - h'/r, all for r > 0."""
    x = kappa * r
    e = np.exp(-x)
    N = -np.expm1(-x) - x * e               # 1 - (1 + x) e^-x
    hp = N / (FOUR_PI * r * r)
    # N - x^2/2 by its series where the difference cancels
    ser = x ** 3 * (-1 / 3 + x * (1 / 8 + x * (-1 / 30 + x * (1 / 144 + x * (-1 / 840 + x / 5760)))))
    Nm = np.where(x < 0.05, ser, N - 0.5 * x * x)
    A_ = Nm / (FOUR_PI * r ** 3)
    B_ = (x * x * e - 3.0 * N) / (FOUR_PI * r ** 3)
    return hp, A_, B_


def hyper_diff_kernel(u, nx, ny, kappa):
    """-d^2/(dn_x dn_y) of (g_Y - g_L) at separation u = x - y (r > 0):
    (nx.ny) h'/r + (u.nx)(u.ny)/r^2 (h'' - h'/r)."""
    u = np.asarray(u, dtype=np.float64)
    r = np.linalg.norm(u, axis=-1)
    hp, _, B_ = _h_derivs(r, kappa)
    un = np.sum(u * nx, axis=-1) * np.sum(u * ny, axis=-1) / (r * r)
    return np.sum(nx * ny, axis=-1) * hp / r + un * B_


def hyper_diff_regular(m: Mesh, s, t, kappa):
    x = m.qpts[s]
    y = m.qpts[t]
    d = x[:, None, :] - y[None, :, :]
    r = np.linalg.norm(d, axis=2)
    ww = m.qw[s][:, None] * m.qw[t][None, :]
    mask = r > 0
    dd = np.where(mask[..., None], d, 1.0)
    k = hyper_diff_kernel(dd, m.normal[s], m.normal[t], kappa)
    return float(np.sum(ww * np.where(mask, k, 0.0)))


def hyper_diff_singular(m: Mesh, s, t, kappa, n_outer: int = 8, n_rem: int = 4):
    """Accurate W_Y - W_L for pairs sharing a vertex: the 1/r part of
    (nx.ny) h'/r, (kappa^2/2)(nx.ny)/(4 pi r), through the closed-form
    triangle potential and the n_outer x n_outer collapsed rule on the test
    triangle; the rest, (nx.ny) A(r) + (u.nx)(u.ny)/r^2 B(r), on the
    n_rem x n_rem collapsed rule on both triangles (on one flat triangle
    u.n = 0 and A(0) = -kappa^3/(12 pi))."""
    s = np.atleast_1d(np.asarray(s))
    t = np.atleast_1d(np.asarray(t))
    tri_s = m.verts[m.tris[s]]
    tri_t = m.verts[m.tris[t]]
    ns, nt = m.normal[s], m.normal[t]
    nn = np.sum(ns * nt, axis=1)
    bo, wo = collapsed_rule(n_outer)
    xo = np.einsum("kj,pjd->pkd", bo, tri_s)
    Wo = wo[None, :] * m.area[s][:, None]
    P = np.sum(Wo * tri_potential(xo, tri_t, nt), axis=1) / FOUR_PI
    out = 0.5 * kappa * kappa * nn * P
    br, wr = collapsed_rule(n_rem)
    xr = np.einsum("kj,pjd->pkd", br, tri_s)
    yr = np.einsum("kj,pjd->pkd", br, tri_t)
    d = xr[:, :, None, :] - yr[:, None, :, :]
    r = np.linalg.norm(d, axis=-1)
    ww = (wr[None, :] * m.area[s][:, None])[:, :, None] * (wr[None, :] * m.area[t][:, None])[:, None, :]
    pos = r > 0
    rr = np.where(pos, r, 1.0)
    _, A_, B_ = _h_derivs(rr, kappa)
    un = (np.einsum("pabd,pd->pab", d, ns) * np.einsum("pabd,pd->pab", d, nt)) / (rr * rr)
    rem = np.where(pos, nn[:, None, None] * A_ + un * B_, -nn[:, None, None] * kappa ** 3 / (12 * math.pi))
    return out + np.sum(ww * rem, axis=(1, 2))


def hyper_diff_operator(m: Mesh, kappa: float, n_outer: int = 8, n_rem: int = 4, chunk: int = 64):
    """Dense W_Y - W_L (T x T): the regular rule on every pair, the singular
    rule on pairs that share a vertex."""
    T = len(m.tris)
    k = m.qpts.shape[1]
    X = m.qpts.reshape(-1, 3)
    Wf = m.qw.reshape(-1)
    nq = np.repeat(m.normal, k, axis=0)
    out = np.zeros((T, T))
    for s0 in range(0, T, chunk):
        s1 = min(T, s0 + chunk)
        Xs = X[s0 * k:s1 * k]
        d = Xs[:, None, :] - X[None, :, :]
        r = np.sqrt(np.einsum("ijd,ijd->ij", d, d))
        mask = r > 0
        dd = np.where(mask[..., None], d, 1.0)
        kk = hyper_diff_kernel(dd, nq[s0 * k:s1 * k][:, None, :], nq[None, :, :], kappa)
        kk = np.where(mask, kk, 0.0)
        ws = Wf[s0 * k:s1 * k]
        out[s0:s1] = (ws[:, None] * kk * Wf[None, :]).reshape(s1 - s0, k, T, k).sum(axis=(1, 3))
    sp = np.array(singular_pairs(m))
    out[sp[:, 0], sp[:, 1]] = hyper_diff_singular(m, sp[:, 0], sp[:, 1], kappa, n_outer, n_rem)
    return out


def system_derivative(m: Mesh, eps1: float, eps2: float, kappa: float, **kw):
    VL, KL = operators(m, 0.0, **kw)
    VY, KY = operators(m, kappa, **kw)
    Wd = hyper_diff_operator(m, kappa, **kw)
    M = np.diag(m.area)
    e21, e12 = eps2 / eps1, eps1 / eps2
    return np.block([[0.5 * (1 + e21) * M - (e21 * KY - KL), VY - VL],
                     [Wd, 0.5 * (1 + e12) * M + (e12 * KY.T - KL.T)]])


def rhs_derivative(m: Mesh, qxyz, q, eps1: float):
    """[b1; b2]: b1 as for the direct formulation; b2_s = int_Ts n_s .
    grad_x sum_k q_k / (4 pi eps1 |x - r_k|)."""
    X = m.qpts.reshape(-1, 3)
    T, k = m.qw.shape
    R = X[:, None, :] - np.asarray(qxyz)[None, :, :]
    d = np.linalg.norm(R, axis=2)
    qq = np.asarray(q)[None, :]
    f1 = (qq / (FOUR_PI * eps1 * d)).sum(axis=1)
    nX = np.repeat(m.normal, k, axis=0)
    f2 = -(qq * np.einsum("ijd,id->ij", R, nX) / (FOUR_PI * eps1 * d ** 3)).sum(axis=1)
    w = m.qw.reshape(-1)
    return np.concatenate([(w * f1).reshape(T, k).sum(axis=1), (w * f2).reshape(T, k).sum(axis=1)])


def solve_derivative(m: Mesh, qxyz, q, eps1=4.0, eps2=80.0, kappa=0.125, **kw):
    A = system_derivative(m, eps1, eps2, kappa, **kw)
    b = rhs_derivative(m, qxyz, q, eps1)
    return np.linalg.solve(A, b), A, b


# ---- exterior derivative formulation (eq:lu) -------------------------------
def system_exterior(m: Mesh, eps1: float, eps2: float, kappa: float, **kw):
    """Exterior derivative formulation (eq:lu, the variant of Lu and
    co-workers), unknowns phi_2 and d phi_2 / dn on the solvent side, with
    e12 = eps1 / eps2:
      [ (1 + e12)/2 M - (K_Y - e12 K_L)   V_Y - V_L                      ]
      [ e12 (W_Y - W_L)                   (1 + e12)/2 M + e12 K'_Y - K'_L ]
    (P0 Galerkin: K' is the transpose of K)."""
    VL, KL = operators(m, 0.0, **kw)
    VY, KY = operators(m, kappa, **kw)
    Wd = hyper_diff_operator(m, kappa, **kw)
    M = np.diag(m.area)
    e12 = eps1 / eps2
    return np.block([[0.5 * (1 + e12) * M - (KY - e12 * KL), VY - VL],
                     [e12 * Wd, 0.5 * (1 + e12) * M + (e12 * KY.T - KL.T)]])


def rhs_exterior(m: Mesh, qxyz, q, eps2: float):
    """Right-hand side of eq:lu: the Coulomb term of the charges and its
    normal derivative, divided by the solvent permittivity eps2."""
    return rhs_derivative(m, qxyz, q, eps2)


def interior_unknowns(x, eps1: float, eps2: float):
    """(phi_1, d phi_1/dn) from the exterior unknowns (phi_2, d phi_2/dn) by
    the interface conditions: the potential is continuous and eps1 d phi_1/dn
    = eps2 d phi_2/dn.  The reaction potential and energy take these."""
    x = np.asarray(x, dtype=np.float64)
    T = len(x) // 2
    return np.concatenate([x[:T], (eps2 / eps1) * x[T:]])


def solve_exterior(m: Mesh, qxyz, q, eps1=4.0, eps2=80.0, kappa=0.125, **kw):
    A = system_exterior(m, eps1, eps2, kappa, **kw)
    b = rhs_exterior(m, qxyz, q, eps2)
    return np.linalg.solve(A, b), A, b


def mass_preconditioned(m: Mesh, A):
    """diag(M, M)^-1 A: the mass-matrix preconditioned operator whose
    eigenvalues the paper studies (for P0 elements the mass matrix is already
    diagonal, so mass lumping changes nothing)."""
    d = np.concatenate([m.area, m.area])
    return A / d[:, None]


def matvec_rows_derivative(m: Mesh, rows, x, eps1=4.0, eps2=80.0, kappa=0.125, formulation="interior",
                           n_outer: int = 8, n_rem: int = 4, chunk: int = 1 << 20):
    """Rows `rows` of A x of the interior (eq:juffer) or exterior (eq:lu)
    derivative formulation for any mesh size: every operator row is a plain
    sum over all trial triangles (regular rule; V, K and K' through the C
    direct sum, K' as n_s . grad of the single-layer potential, W_Y - W_L in
    NumPy over source chunks), and the pairs that share a vertex take the
    singular rule (K' from the transposed K pair).  Returns (len(rows), 2)."""
    from . import direct as Dd
    T = len(m.tris)
    k = m.qpts.shape[1]
    rows = np.asarray(rows)
    u, v = x[:T], x[T:]
    Y = m.qpts.reshape(-1, 3)
    W = m.qw.reshape(-1)
    n_rep = np.repeat(m.normal, k, axis=0)
    uu = np.repeat(u, k) * W
    vv = np.repeat(v, k) * W
    tgt = m.qpts[rows].reshape(-1, 3)
    wt = m.qw[rows].reshape(-1)
    nt = np.repeat(m.normal[rows], k, axis=0)
    by_row = {int(s_): np.nonzero(np.isin(m.tris, m.tris[s_]).any(axis=1))[0] for s_ in rows}
    ops = {}
    for kern, kap in (("laplace", 0.0), ("yukawa", kappa)):
        Kx = np.zeros(len(tgt))
        for d in range(3):
            _, g = Dd.direct(tgt, Y, uu * n_rep[:, d], kern, kap)
            Kx -= g[:, d]
        Vx, gv = Dd.direct(tgt, Y, vv, kern, kap)
        Kpx = np.sum(nt * gv, axis=1)
        Kr = (wt * Kx).reshape(len(rows), k).sum(axis=1)
        Vr = (wt * Vx).reshape(len(rows), k).sum(axis=1)
        Kpr = (wt * Kpx).reshape(len(rows), k).sum(axis=1)
        for i, s_ in enumerate(rows):
            ts = by_row[int(s_)]
            Vs, Ks = singular_entries(m, np.full(len(ts), s_), ts, kap, n_outer, n_rem)
            _, Kts = singular_entries(m, ts, np.full(len(ts), s_), kap, n_outer, n_rem)
            for j, t_ in enumerate(ts):
                Vreg, Kreg = regular_entries(m, s_, t_, kap)
                _, Ktreg = regular_entries(m, t_, s_, kap)
                Vr[i] += (Vs[j] - Vreg) * v[t_]
                Kr[i] += (Ks[j] - Kreg) * u[t_]
                Kpr[i] += (Kts[j] - Ktreg) * v[t_]
        ops[kern] = (Vr, Kr, Kpr)
    # W_Y - W_L: regular rule over all quadrature points, then the singular pairs
    Wr = np.zeros(len(rows))
    for i, s_ in enumerate(rows):
        acc = 0.0
        for a in range(k):
            xa = m.qpts[s_, a]
            tot = 0.0
            for c0 in range(0, len(Y), chunk):
                dd = xa[None, :] - Y[c0:c0 + chunk]
                r = np.linalg.norm(dd, axis=1)
                mask = r > 0
                dd = np.where(mask[:, None], dd, 1.0)
                kv = hyper_diff_kernel(dd, m.normal[s_], n_rep[c0:c0 + chunk], kappa)
                tot += float(np.sum(np.where(mask, kv, 0.0) * uu[c0:c0 + chunk]))
            acc += m.qw[s_, a] * tot
        ts = by_row[int(s_)]
        Ws = hyper_diff_singular(m, np.full(len(ts), s_), ts, kappa, n_outer, n_rem)
        for j, t_ in enumerate(ts):
            acc += (Ws[j] - hyper_diff_regular(m, s_, t_, kappa)) * u[t_]
        Wr[i] = acc
    VL, KL, KpL = ops["laplace"]
    VY, KY, KpY = ops["yukawa"]
    e12, e21 = eps1 / eps2, eps2 / eps1
    A_ = m.area[rows]
    out = np.zeros((len(rows), 2))
    if formulation == "interior":
        out[:, 0] = 0.5 * (1 + e21) * A_ * u[rows] - (e21 * KY - KL) + (VY - VL)
        out[:, 1] = Wr + 0.5 * (1 + e12) * A_ * v[rows] + (e12 * KpY - KpL)
    elif formulation == "exterior":
        out[:, 0] = 0.5 * (1 + e12) * A_ * u[rows] - (KY - e12 * KL) + (VY - VL)
        out[:, 1] = e12 * Wr + 0.5 * (1 + e12) * A_ * v[rows] + (e12 * KpY - KpL)
    else:
        raise ValueError(formulation)
    return out
