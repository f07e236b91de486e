"""Dense P1 Galerkin oracle for the exterior derivative formulation (eq:lu)
of the linearised Poisson-Boltzmann interface problem (Methods: the
derivative formulations and their operators; Results: the exterior variant
with piecewise-linear elements and mass-matrix preconditioning).

TEST INFRASTRUCTURE ONLY (see the package docstring).  FP64, dense, small
meshes.

Discretisation (readings where the paper is silent):
  * Continuous piecewise-linear trial and test functions: the hat function
    phi_i of vertex i; on triangle t with vertices (t0, t1, t2) it is the
    barycentric coordinate lambda_a of the corner a with t_a = i.  Unknowns
    per vertex: u_i (the solvent-side potential phi_2) and v_i (its normal
    derivative).
  * Quadrature-point densities interpolate the vertex values:
    u(x_j) = sum_a lambda_a(xi_j) u_{t_a}; test integrals weight the
    quadrature-point fields by W_j lambda_a(xi_j) and add them into vertex t_a.
  * Operators (i, j vertices): V_ij = int int phi_i g phi_j, K_ij with
    dg/dn_y, K' = K^T (dg/dn_x, the transposed pair), W_Y - W_L as in the P0
    oracle, M_ij = int phi_i phi_j (on a triangle of area A: A/12 times
    2 on the diagonal and 1 off it).
  * Pairs of triangles that share no vertex: the regular rule on both
    triangles.  Pairs that share a vertex: 3 x 3 blocks with the Laplace part
    of the inner integral in closed form for a linear density (below), the
    outer integral on the collapsed rule, the bounded Yukawa remainders on
    the collapsed rule on both triangles, exactly as the P0 oracle but with
    the hat-function weights.
  * Closed form for a linear density on a flat triangle T seen from x, with
    d = n.(x - v0), rho = x - d n, R = |x - y|, lambda linear on T:
      int_T lambda(y)/R dy     = lambda(rho) P + grad(lambda) . G
      int_T lambda(y) d/R^3 dy = lambda(rho) D + d grad(lambda) . H
    P and D are the P0 closed forms (uniform potential, minus the solid
    angle); G = int_T (y - rho)/R dy and H = int_T (y - rho)/R^3 dy follow
    from the divergence theorem in the plane of T, since (y - rho)/R is the
    in-plane gradient of R and (y - rho)/R^3 that of -1/R:
      G = sum over edges of m_e int_e R dl,   H = -sum over edges of m_e int_e dl/R
    (m_e the outward in-plane normal of the edge; along an edge R^2 = l^2 + c^2
    with c^2 = t0^2 + d^2, so int R dl = (l R + c^2 log(l + R))/2 and
    int dl/R = log(l + R) between the edge's end coordinates).
  * Preconditioner: the lumped mass matrix diag(Ml, Ml), Ml_i = sum over the
    triangles at vertex i of A/3 (the row sums of M).
  * The reaction potential and the energy take the interior unknowns
    (u, (eps2/eps1) v) interpolated to the quadrature points.
"""
from __future__ import annotations

import numpy as np

from . import bem
from .bem import FOUR_PI, Mesh


# ---------------------------------------------------------------------------
# linear-density closed forms
# ---------------------------------------------------------------------------
def _log_ratio(lp, lm, Rp, Rm, c2):
    """log((lp + Rp) / (lm + Rm)) with R = sqrt(l^2 + c2), lp > lm, in a
    form without cancellation: for l < 0, l + R = c2 / (R - l)."""
    with np.errstate(divide="ignore", invalid="ignore"):
        both_pos = np.log((lp + Rp) / (lm + Rm))
        both_neg = np.log((Rm - lm) / (Rp - lp))
        mixed = np.log((lp + Rp) * (Rm - lm) / c2)
    return np.where(lm >= 0, both_pos, np.where(lp <= 0, both_neg, mixed))


def linear_moments(x, tri, n):
    """(G, H): int_T (y - rho)/R dy and int_T (y - rho)/R^3 dy for the flat
    triangle T with unit normal n seen from x (see the module notes).
    Batched like bem.tri_potential: x (..., k, 3) -> (..., k, 3) each.  H is
    returned multiplied by d (it only enters as d H), which is finite
    wherever x is off the triangle's edges."""
    x = np.asarray(x, dtype=np.float64)
    tri = np.asarray(tri, dtype=np.float64)
    n = np.asarray(n, dtype=np.float64)
    nn = n[..., None, :]
    d = np.sum((x - tri[..., 0:1, :]) * nn, axis=-1)
    rho = x - d[..., None] * nn
    G = np.zeros(x.shape)
    dH = np.zeros(x.shape)
    for i in range(3):
        a = tri[..., i:i + 1, :]
        b = tri[..., (i + 1) % 3:(i + 1) % 3 + 1, :]
        L = np.linalg.norm(b - a, axis=-1)
        lh = (b - a) / L[..., None]
        m_e = np.cross(lh, nn)                  # outward in-plane normal (counter-clockwise T)
        t0 = np.sum((a - rho) * m_e, axis=-1)
        lp = np.sum((b - rho) * lh, axis=-1)
        lm = np.sum((a - rho) * lh, axis=-1)
        Rp = np.linalg.norm(x - b, axis=-1)
        Rm = np.linalg.norm(x - a, axis=-1)
        c2 = t0 * t0 + d * d
        lg = _log_ratio(lp, lm, Rp, Rm, c2)
        tiny = c2 <= (1e-14 * L) ** 2
        iR = 0.5 * (lp * Rp - lm * Rm + np.where(tiny, 0.0, c2 * lg))
        G += iR[..., None] * m_e
        dH -= np.where(d == 0, 0.0, d * np.where(tiny, 0.0, lg))[..., None] * m_e
    return G, dH


def hat_gradients(tri, n):
    """Gradients of the barycentric coordinates of the triangle(s) tri
    (..., 3, 3) with unit normal n: grad lambda_a = n x (v_{a+2} - v_{a+1}) / (2 A)."""
    tri = np.asarray(tri, dtype=np.float64)
    n = np.asarray(n, dtype=np.float64)
    area2 = np.linalg.norm(np.cross(tri[..., 1, :] - tri[..., 0, :], tri[..., 2, :] - tri[..., 0, :]), axis=-1)
    g = [np.cross(n, tri[..., (a + 2) % 3, :] - tri[..., (a + 1) % 3, :]) / area2[..., None] for a in range(3)]
    return np.stack(g, axis=-2)               # (..., 3 corners, 3)


def _hat_at(y, tri, grads):
    """lambda_a(y) for points y (..., k, 3) in the plane of tri: (..., k, 3 corners)."""
    rel = y - tri[..., 0:1, :]
    lam = np.einsum("...kd,...ad->...ka", rel, grads)
    lam[..., 0] += 1.0
    return lam


# ---------------------------------------------------------------------------
# 3 x 3 blocks of the pairs that share a vertex
# ---------------------------------------------------------------------------
def singular_blocks(m: Mesh, s, t, kappa, n_outer: int = 8, n_rem: int = 4):
    """Accurate (V, K, W_Y - W_L) 3 x 3 blocks [corner of s][corner of t]
    for pairs (s, t) that share a vertex: arrays (P, 3, 3) each."""
    s = np.atleast_1d(np.asarray(s))
    t = np.atleast_1d(np.asarray(t))
    tri_s = m.verts[m.tris[s]]
    tri_t = m.verts[m.tris[t]]
    ns, nt = m.normal[s], m.normal[t]
    gt = hat_gradients(tri_t, nt)                             # (P, 3, 3)
    bo, wo = bem.collapsed_rule(n_outer)
    xo = np.einsum("kj,pjd->pkd", bo, tri_s)                  # (P, k, 3)
    Wo = wo[None, :] * m.area[s][:, None]                     # (P, k)
    P0 = bem.tri_potential(xo, tri_t, nt)                     # (P, k)
    D0 = bem.tri_dlp(xo, tri_t, nt)
    G, dH = linear_moments(xo, tri_t, nt)
    d = np.sum((xo - tri_t[:, 0:1, :]) * nt[:, None, :], axis=-1)
    rho = xo - d[..., None] * nt[:, None, :]
    lam_rho = _hat_at(rho, tri_t, gt)                         # (P, k, 3)
    inner_v = lam_rho * P0[..., None] + np.einsum("pkd,pbd->pkb", G, gt)
    inner_k = lam_rho * D0[..., None] + np.einsum("pkd,pbd->pkb", dH, gt)
    same = (s == t)[:, None, None]
    Vb = np.einsum("pk,ka,pkb->pab", Wo, bo, inner_v) / FOUR_PI
    Kb = np.where(same, 0.0, np.einsum("pk,ka,pkb->pab", Wo, bo, inner_k) / FOUR_PI)
    nn = np.sum(ns * nt, axis=1)
    Wb = 0.5 * kappa * kappa * nn[:, None, None] * Vb
    # bounded remainders on the collapsed rule on both triangles
    br, wr = bem.collapsed_rule(n_rem)
    xr = np.einsum("kj,pjd->pkd", br, tri_s)
    yr = np.einsum("kj,pjd->pkd", br, tri_t)
    dd = xr[:, :, None, :] - yr[:, None, :, :]
    r = np.linalg.norm(dd, axis=-1)
    ww = (wr[None, :] * m.area[s][:, None])[:, :, None] * (wr[None, :] * m.area[t][:, None])[:, None, :]
    pos = r > 0
    rr = np.where(pos, r, 1.0)
    _, A_, B_ = bem._h_derivs(rr, kappa)
    un = (np.einsum("pabd,pd->pab", dd, ns) * np.einsum("pabd,pd->pab", dd, nt)) / (rr * rr)
    remW = np.where(pos, nn[:, None, None] * A_ + un * B_, -nn[:, None, None] * kappa ** 3 / (12 * np.pi))
    Wb = Wb + np.einsum("pij,ia,jb->pab", ww * remW, br, br)
    if kappa > 0:
        kr = kappa * rr
        dn = np.einsum("pijd,pd->pij", dd, nt)
        remV = np.where(pos, np.expm1(-kr) / (FOUR_PI * rr), -kappa / FOUR_PI)
        remK = np.where(pos, dn * ((1 + kr) * np.exp(-kr) - 1.0) / (FOUR_PI * rr ** 3), 0.0)
        Vb = Vb + np.einsum("pij,ia,jb->pab", ww * remV, br, br)
        Kb = Kb + np.where(same, 0.0, np.einsum("pij,ia,jb->pab", ww * remK, br, br))
    return Vb, Kb, Wb


def regular_blocks(m: Mesh, s, t, kappa):
    """The regular-rule (quadrature-point) 3 x 3 blocks of V, K and W_Y - W_L
    for pairs (s, t), zero-distance point pairs left out."""
    s = np.atleast_1d(np.asarray(s))
    t = np.atleast_1d(np.asarray(t))
    bary, _ = bem.regular_rule(m.qpts.shape[1])
    x, y = m.qpts[s], m.qpts[t]                               # (P, k, 3)
    dd = x[:, :, None, :] - y[:, None, :, :]
    r = np.linalg.norm(dd, axis=-1)
    pos = r > 0
    rr = np.where(pos, r, 1.0)
    ww = m.qw[s][:, :, None] * m.qw[t][:, None, :]
    e = np.exp(-kappa * rr)
    g = np.where(pos, e / (FOUR_PI * rr), 0.0)
    dn = np.einsum("pijd,pd->pij", dd, m.normal[t])
    kk = np.where(pos, dn * (1 + kappa * rr) * e / (FOUR_PI * rr ** 3), 0.0)
    ddm = np.where(pos[..., None], dd, 1.0)
    hw = np.where(pos, bem.hyper_diff_kernel(ddm, m.normal[s][:, None, None, :], m.normal[t][:, None, None, :],
                                             kappa), 0.0)
    blk = lambda f: np.einsum("pij,ia,jb->pab", ww * f, bary, bary)
    return blk(g), blk(kk), blk(hw)


# ---------------------------------------------------------------------------
# dense operators
# ---------------------------------------------------------------------------
def interpolation(m: Mesh):
    """L (N, nv): quadrature-point values from vertex values,
    L[(t, j), t_a] = lambda_a(xi_j)."""
    T, k = m.qw.shape
    nv = len(m.verts)
    bary, _ = bem.regular_rule(k)
    L = np.zeros((T * k, nv))
    for a in range(3):
        np.add.at(L, (np.arange(T * k), np.repeat(m.tris[:, a], k)), np.tile(bary[:, a], T))
    return L


def mass(m: Mesh):
    nv = len(m.verts)
    M = np.zeros((nv, nv))
    loc = np.array([[2.0, 1.0, 1.0], [1.0, 2.0, 1.0], [1.0, 1.0, 2.0]]) / 12.0
    for a in range(3):
        for b in range(3):
            np.add.at(M, (m.tris[:, a], m.tris[:, b]), m.area * loc[a, b])
    return M


def lumped_mass(m: Mesh):
    Ml = np.zeros(len(m.verts))
    for a in range(3):
        np.add.at(Ml, m.tris[:, a], m.area / 3.0)
    return Ml


def _add_blocks(out, m: Mesh, s, t, blocks):
    for a in range(3):
        for b in range(3):
            np.add.at(out, (m.tris[s, a], m.tris[t, b]), blocks[:, a, b])


def operators(m: Mesh, kappa: float, n_outer: int = 8, n_rem: int = 4, chunk: int = 256):
    """Dense P1 V, K and W_Y - W_L (nv x nv) for one kernel (W only
    meaningful for kappa > 0): L^T (quadrature-point sums) L, then the pairs
    that share a vertex swap their regular blocks for accurate ones."""
    X = m.qpts.reshape(-1, 3)
    Wf = m.qw.reshape(-1)
    k = m.qpts.shape[1]
    nq = np.repeat(m.normal, k, axis=0)
    L = interpolation(m)
    nv = len(m.verts)
    V, K, Wd = np.zeros((nv, nv)), np.zeros((nv, nv)), np.zeros((nv, nv))
    for i0 in range(0, len(X), chunk):
        i1 = min(len(X), i0 + chunk)
        dd = X[i0:i1, None, :] - X[None, :, :]
        r = np.linalg.norm(dd, axis=-1)
        pos = r > 0
        rr = np.where(pos, r, 1.0)
        e = np.exp(-kappa * rr)
        g = np.where(pos, e / (FOUR_PI * rr), 0.0)
        kk = np.where(pos, np.einsum("ijd,jd->ij", dd, nq) * (1 + kappa * rr) * e / (FOUR_PI * rr ** 3), 0.0)
        ddm = np.where(pos[..., None], dd, 1.0)
        hw = np.where(pos, bem.hyper_diff_kernel(ddm, nq[i0:i1, None, :], nq[None, :, :], kappa), 0.0)
        wl = (Wf[i0:i1, None] * L[i0:i1]).T                    # (nv, rows)
        V += wl @ (g * Wf[None, :]) @ L
        K += wl @ (kk * Wf[None, :]) @ L
        Wd += wl @ (hw * Wf[None, :]) @ L
    sp = np.array(bem.singular_pairs(m))
    s, t = sp[:, 0], sp[:, 1]
    Vs, Ks, Ws = singular_blocks(m, s, t, kappa, n_outer, n_rem)
    Vr, Kr, Wr = regular_blocks(m, s, t, kappa)
    _add_blocks(V, m, s, t, Vs - Vr)
    _add_blocks(K, m, s, t, Ks - Kr)
    _add_blocks(Wd, m, s, t, Ws - Wr)
    return V, K, Wd


def system_exterior(m: Mesh, eps1: float, eps2: float, kappa: float, **kw):
    """eq:lu on P1 elements, e12 = eps1 / eps2 (2 nv x 2 nv):
      [ (1 + e12)/2 M - (K_Y - e12 K_L)   V_Y - V_L                      ]
      [ e12 (W_Y - W_L)                   (1 + e12)/2 M + e12 K'_Y - K'_L ]"""
    VL, KL, _ = operators(m, 0.0, **kw)
    VY, KY, Wd = operators(m, kappa, **kw)
    M = mass(m)
    e12 = eps1 / eps2
    return np.block([[0.5 * (1 + e12) * M - (KY - e12 * KL), VY - VL],
                     [e12 * Wd, 0.5 * (1 + e12) * M + (e12 * KY.T - KL.T)]])


def rhs_exterior(m: Mesh, qxyz, q, eps2: float):
    """The Coulomb potential of the charges over eps2 and its normal
    derivative, tested with the hat functions."""
    X = m.qpts.reshape(-1, 3)
    T, k = m.qw.shape
    R = X[:, None, :] - np.asarray(qxyz, dtype=np.float64)[None, :, :]
    d = np.linalg.norm(R, axis=2)
    qq = np.asarray(q, dtype=np.float64)[None, :]
    f1 = (qq / (FOUR_PI * eps2 * d)).sum(axis=1)
    nX = np.repeat(m.normal, k, axis=0)
    f2 = -(qq * np.einsum("ijd,id->ij", R, nX) / (FOUR_PI * eps2 * d ** 3)).sum(axis=1)
    L = interpolation(m)
    w = m.qw.reshape(-1)
    return np.concatenate([L.T @ (w * f1), L.T @ (w * f2)])


def solve_exterior(m: Mesh, qxyz, q, eps1=4.0, eps2=80.0, kappa=0.125, **kw):
    A = system_exterior(m, eps1, eps2, kappa, **kw)
    b = rhs_exterior(m, qxyz, q, eps2)
    return np.linalg.solve(A, b), A, b


def reaction_potential(m: Mesh, x, qxyz, eps1=4.0, eps2=80.0):
    """Reaction potential at qxyz from the exterior P1 unknowns x = (u, v):
    the interior unknowns (u, (eps2/eps1) v) at the quadrature points, then
    the same quadrature sum as the P0 oracle."""
    nv = len(m.verts)
    L = interpolation(m)
    uq = L @ x[:nv]
    vq = (eps2 / eps1) * (L @ x[nv:])
    W = m.qw.reshape(-1)
    k = m.qpts.shape[1]
    Y = m.qpts.reshape(-1, 3)
    nY = np.repeat(m.normal, k, axis=0)
    R = np.asarray(qxyz, dtype=np.float64)[:, None, :] - Y[None, :, :]
    r = np.linalg.norm(R, axis=2)
    g = 1.0 / (FOUR_PI * r)
    dgdn = np.einsum("kjd,jd->kj", R, nY) / (FOUR_PI * r ** 3)
    return -dgdn @ (W * uq) + g @ (W * vq)


def energy(m: Mesh, x, qxyz, q, eps1=4.0, eps2=80.0):
    phi = reaction_potential(m, x, qxyz, eps1, eps2)
    return 0.5 * float(np.dot(q, phi)) * FOUR_PI * bem.KCAL_PER_MOL


def lumped_preconditioned(m: Mesh, A):
    """diag(Ml, Ml)^-1 A."""
    d = np.concatenate([lumped_mass(m)] * 2)
    return A / d[:, None]


def matvec_rows(m: Mesh, rows, x, eps1=4.0, eps2=80.0, kappa=0.125, n_outer: int = 8, n_rem: int = 4,
                chunk: int = 1 << 23):
    """Rows `rows` (vertex indices) of the P1 exterior system times x for any
    mesh size, (len(rows), 2).  Each row is a sum over the triangle corners
    at the vertex: the fields of all quadrature-point sources (the vertex
    values interpolated; V, K and K' through the C direct sum, K' as n_s .
    grad of the single-layer potential, W_Y - W_L in NumPy over source
    chunks) weighted by W_j lambda_a(xi_j), the singular pairs' blocks
    swapped for accurate ones (K' from the transposed pair), and the mass
    matrix.  Every vertex must lie on a triangle."""
    from . import direct as Dd
    nv = len(m.verts)
    T, k = m.qw.shape
    u, v = x[:nv], x[nv:]
    bary, _ = bem.regular_rule(k)
    uq = np.einsum("ja,ta->tj", bary, u[m.tris]).reshape(-1)
    vq = np.einsum("ja,ta->tj", bary, v[m.tris]).reshape(-1)
    Y = m.qpts.reshape(-1, 3)
    W = m.qw.reshape(-1)
    n_rep = np.repeat(m.normal, k, axis=0)
    uu, vv = W * uq, W * vq
    e12 = eps1 / eps2
    out = np.zeros((len(rows), 2))
    for r_i, vi in enumerate(np.asarray(rows)):
        ss, aa = np.nonzero(m.tris == vi)                       # corners (s, a) at the vertex
        tgt = m.qpts[ss].reshape(-1, 3)
        wt = (m.qw[ss] * bary[:, aa].T).reshape(-1)              # W_j lambda_a(xi_j)
        nt = np.repeat(m.normal[ss], k, axis=0)
        fields = {}
        for kern, kap in (("laplace", 0.0), ("yukawa", kappa)):
            Kx = np.zeros(len(tgt))
            for d in range(3):
                _, g = Dd.direct(tgt, Y, uu * n_rep[:, d], kern, kap)
                Kx -= g[:, d]
            Vx, gv = Dd.direct(tgt, Y, vv, kern, kap)
            fields[kern] = [float(wt @ Vx), float(wt @ Kx), float(wt @ np.sum(nt * gv, axis=1))]
        # W_Y - W_L: all of the row's targets against a chunk of sources at a time
        tot = np.zeros(len(tgt))
        step = max(1, chunk // len(tgt))
        for c0 in range(0, len(Y), step):
            dd = tgt[:, None, :] - Y[None, c0:c0 + step]
            r = np.linalg.norm(dd, axis=-1)
            pos = r > 0
            dd = np.where(pos[..., None], dd, 1.0)
            kv = bem.hyper_diff_kernel(dd, nt[:, None, :], n_rep[None, c0:c0 + step], kappa)
            tot += np.where(pos, kv, 0.0) @ uu[c0:c0 + step]
        Wr = float(wt @ tot)
        mu = mv = 0.0
        for s_, a_ in zip(ss, aa):
            ts = np.nonzero(np.isin(m.tris, m.tris[s_]).any(axis=1))[0]
            S = np.full(len(ts), s_)
            ut, vt = u[m.tris[ts]], v[m.tris[ts]]                 # (P, 3) trial values
            for kern, kap in (("laplace", 0.0), ("yukawa", kappa)):
                Vs, Ks, _ = singular_blocks(m, S, ts, kap, n_outer, n_rem)
                Vr, Kr, _ = regular_blocks(m, S, ts, kap)
                _, Kts, _ = singular_blocks(m, ts, S, kap, n_outer, n_rem)
                _, Ktr, _ = regular_blocks(m, ts, S, kap)
                fields[kern][0] += float(np.sum((Vs - Vr)[:, a_, :] * vt))
                fields[kern][1] += float(np.sum((Ks - Kr)[:, a_, :] * ut))
                fields[kern][2] += float(np.sum((Kts - Ktr)[:, :, a_] * vt))
            _, _, Ws = singular_blocks(m, S, ts, kappa, n_outer, n_rem)
            _, _, Wreg = regular_blocks(m, S, ts, kappa)
            Wr += float(np.sum((Ws - Wreg)[:, a_, :] * ut))
            loc = m.area[s_] / 12.0
            mu += loc * (u[vi] + u[m.tris[s_]].sum())
            mv += loc * (v[vi] + v[m.tris[s_]].sum())
        VL, KL, KpL = fields["laplace"]
        VY, KY, KpY = fields["yukawa"]
        out[r_i, 0] = 0.5 * (1 + e12) * mu - (KY - e12 * KL) + (VY - VL)
        out[r_i, 1] = e12 * Wr + 0.5 * (1 + e12) * mv + (e12 * KpY - KpL)
    return out


def energy_direct(m: Mesh, x, qxyz, q, eps1=4.0, eps2=80.0):
    """energy() through the C direct sum for meshes too large for the dense
    kernel matrix: the interior unknowns interpolated to the quadrature
    points, then the P0 oracle's direct-sum reaction potential."""
    nv = len(m.verts)
    k = m.qpts.shape[1]
    bary, _ = bem.regular_rule(k)
    # per-triangle "P0" arrays holding the interpolated quadrature values
    uq = np.einsum("ja,ta->tj", bary, x[:nv][m.tris])
    vq = (eps2 / eps1) * np.einsum("ja,ta->tj", bary, x[nv:][m.tris])
    from . import direct as Dd
    Y = m.qpts.reshape(-1, 3)
    W = m.qw.reshape(-1)
    nY = np.repeat(m.normal, k, axis=0)
    tgt = np.ascontiguousarray(qxyz, dtype=np.float64).reshape(-1, 3)
    phi, _ = Dd.direct(tgt, Y, W * vq.reshape(-1))
    for d in range(3):
        _, g = Dd.direct(tgt, Y, W * uq.reshape(-1) * nY[:, d])
        phi += g[:, d]
    return 0.5 * float(np.dot(q, phi)) * FOUR_PI * bem.KCAL_PER_MOL
