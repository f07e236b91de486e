"""Pins of the P1 exterior-formulation oracle: the linear-density closed
forms against brute-force quadrature, the hat-function blocks summing to the
P0 entries, Gauss's theorem and Green's identity for a linear harmonic
field, and the Kirkwood solvation energy with first-order convergence."""
import math

import numpy as np
import pytest

import synth
from oracle import analytic as A
from oracle import bem
from oracle import bem_p1 as P

KAPPA = 0.125


def _subdivided(tri, f, N=32):
    """int_T f(y) dy on N^2 congruent sub-triangles with the 6-point rule
    (f: (k, 3) -> (k, ...))."""
    bary, w = bem.regular_rule(6)
    out = 0.0
    for i in range(N):
        for j in range(N - i):
            cells = [[(i, j), (i + 1, j), (i, j + 1)]]
            if i + j < N - 1:
                cells.append([(i + 1, j), (i + 1, j + 1), (i, j + 1)])
            for c in cells:
                pts = np.array([tri[0] + (a / N) * (tri[1] - tri[0]) + (b / N) * (tri[2] - tri[0]) for a, b in c])
                ar = 0.5 * np.linalg.norm(np.cross(pts[1] - pts[0], pts[2] - pts[0]))
                out = out + ar * np.tensordot(w, f(bary @ pts), axes=(0, 0))
    return out


def test_linear_density_closed_forms_against_brute_force():
    tri = np.array([[0.0, 0.0, 0.0], [1.3, 0.1, 0.0], [0.2, 0.9, 0.1]])
    n = np.cross(tri[1] - tri[0], tri[2] - tri[0])
    n /= np.linalg.norm(n)
    rng = np.random.default_rng(31)
    c = tri.mean(axis=0)
    # above and below the triangle, and in its plane outside it
    x = np.concatenate([c + rng.normal(0, 1.0, (6, 3)) + 1.5 * n, c - 0.6 * n + rng.normal(0, 0.2, (3, 3)),
                        tri[0] + np.array([[-0.8, -0.5, 0.0], [2.0, 1.5, 0.1]])])
    x[-2:] -= ((x[-2:] - tri[0]) @ n)[:, None] * n
    gr = P.hat_gradients(tri, n)
    G, dH = P.linear_moments(x, tri, n)
    P0, D0 = bem.tri_potential(x, tri, n), bem.tri_dlp(x, tri, n)
    d = (x - tri[0]) @ n
    lam_rho = P._hat_at((x - d[:, None] * n)[None], tri[None], gr[None])[0]
    for b in range(3):
        lam = lambda y: (b == 0) + (y - tri[0]) @ gr[b]
        R = lambda y: np.linalg.norm(x[None] - y[:, None], axis=2)
        bv = _subdivided(tri, lambda y: lam(y)[:, None] / R(y))
        bk = _subdivided(tri, lambda y: lam(y)[:, None] * ((x[None] - y[:, None]) @ n) / R(y) ** 3)
        np.testing.assert_allclose(lam_rho[:, b] * P0 + G @ gr[b], bv, rtol=1e-9)
        np.testing.assert_allclose(lam_rho[:, b] * D0 + dH @ gr[b], bk, rtol=1e-7, atol=1e-12)


def test_hat_gradients_and_mass():
    v, t = synth.octa_sphere(1, 2.0)
    m = bem.make_mesh(v, t, 3)
    gr = P.hat_gradients(m.verts[m.tris], m.normal)
    for a in range(3):
        for b in range(3):
            # lambda_a(v_b) = delta_ab through lambda_a(y) = [a == 0] + grad . (y - v0)
            val = (a == 0) + np.sum(gr[:, a] * (m.verts[m.tris[:, b]] - m.verts[m.tris[:, 0]]), axis=1)
            np.testing.assert_allclose(val, float(a == b), atol=1e-13)
    M = P.mass(m)
    np.testing.assert_allclose(M, M.T)
    np.testing.assert_allclose(M.sum(axis=1), P.lumped_mass(m), rtol=1e-14)
    assert M.sum() == pytest.approx(m.area.sum(), rel=1e-14)
    assert np.linalg.eigvalsh(M).min() > 0


@pytest.mark.parametrize("kappa", [0.0, KAPPA])
def test_hat_blocks_sum_to_the_p0_entries(kappa):
    """sum_a lambda_a = 1 on both triangles: every 3 x 3 block sums to the P0
    entry of the same pair (accurate and regular rules), and the assembled
    P1 operators sum to the P0 operators' totals."""
    v, t = synth.octa_sphere(2, 4.0)
    m = bem.make_mesh(v, t, 3)
    sp = np.array(bem.singular_pairs(m))
    s, t_ = sp[:, 0], sp[:, 1]
    Vb, Kb, Wb = P.singular_blocks(m, s, t_, kappa)
    V0, K0 = bem.singular_entries(m, s, t_, kappa)
    np.testing.assert_allclose(Vb.sum(axis=(1, 2)), V0, rtol=1e-12, atol=1e-15 * np.abs(V0).max())
    np.testing.assert_allclose(Kb.sum(axis=(1, 2)), K0, rtol=1e-12, atol=1e-14 * np.abs(K0).max())
    Vr, Kr, _ = P.regular_blocks(m, s, t_, kappa)
    reg = np.array([bem.regular_entries(m, a, b, kappa) for a, b in sp])
    np.testing.assert_allclose(Vr.sum(axis=(1, 2)), reg[:, 0], rtol=1e-12)
    V1, K1, W1 = P.operators(m, kappa)
    V0d, K0d = bem.operators(m, kappa)
    assert V1.sum() == pytest.approx(V0d.sum(), rel=1e-12)
    assert K1.sum() == pytest.approx(K0d.sum(), rel=1e-12, abs=1e-12)
    if kappa > 0:
        W0 = bem.hyper_diff_singular(m, s, t_, kappa)
        np.testing.assert_allclose(Wb.sum(axis=(1, 2)), W0, rtol=1e-12, atol=1e-15 * np.abs(W0).max())
        assert W1.sum() == pytest.approx(bem.hyper_diff_operator(m, kappa).sum(), rel=1e-12)
    # Galerkin with a symmetric kernel: V symmetric up to quadrature error
    assert np.abs(V1 - V1.T).max() < 1e-5 * np.abs(V1).max()


def test_double_layer_of_a_constant_is_minus_half():
    v, t = synth.octa_sphere(2, 4.0)
    m = bem.make_mesh(v, t, 3)
    _, K, _ = P.operators(m, 0.0)
    assert np.abs(K.sum(axis=1) / P.lumped_mass(m) + 0.5).max() < 1e-3


def _v_hat_test_p0_trial(m):
    """Laplace single layer with hat test functions and piecewise-constant
    trial functions: (nv, T), the singular pairs through the block sums over
    the trial corners."""
    X = m.qpts.reshape(-1, 3)
    Wf = m.qw.reshape(-1)
    T, k = m.qw.shape
    L = P.interpolation(m)
    E = np.kron(np.eye(T), np.ones((k, 1)))
    r = np.linalg.norm(X[:, None] - X[None], axis=-1)
    g = np.where(r > 0, 1.0 / (4 * math.pi * np.where(r > 0, r, 1.0)), 0.0)
    Vm = (Wf[:, None] * L).T @ (g * Wf[None, :]) @ E
    sp = np.array(bem.singular_pairs(m))
    Vs, _, _ = P.singular_blocks(m, sp[:, 0], sp[:, 1], 0.0)
    Vr, _, _ = P.regular_blocks(m, sp[:, 0], sp[:, 1], 0.0)
    for a in range(3):
        np.add.at(Vm, (m.tris[sp[:, 0], a], sp[:, 1]), (Vs - Vr)[:, a, :].sum(axis=-1))
    return Vm


def test_green_identity_for_a_linear_field():
    """u(y) = a . y is harmonic inside the polyhedron and exactly in the P1
    space; Green's representation on the boundary gives M u / 2 + K_L u =
    V_L (a . n) with the piecewise-constant normal derivative (this exercises
    the linear-density part of K)."""
    a = np.array([0.3, -0.8, 0.5])
    v, t = synth.octa_sphere(2, 4.0, center=(0.5, -0.2, 0.1))
    m = bem.make_mesh(v, t, 3)
    _, KL, _ = P.operators(m, 0.0)
    M = P.mass(m)
    u = m.verts @ a
    res = 0.5 * M @ u + KL @ u - _v_hat_test_p0_trial(m) @ (m.normal @ a)
    assert np.linalg.norm(res) < 1e-3 * np.linalg.norm(M @ u)


def test_exterior_p1_kirkwood_convergence_and_spectrum():
    """Kirkwood sphere: the P1 exterior formulation's energy converges at
    order 1 (the flat-triangle geometry error), and under the lumped mass
    preconditioner its eigenvalues stay near (1 + eps1/eps2)/2."""
    ref = A.kirkwood_energy(4.0, [1, 1, 1], [1.0], 4.0, 80.0, KAPPA)
    err = []
    for lev in (2, 3):
        v, t = synth.octa_sphere(lev, 4.0)
        m = bem.make_mesh(v, t, 3)
        x, Am, _ = P.solve_exterior(m, [[1, 1, 1]], [1.0])
        err.append(abs(P.energy(m, x, [[1, 1, 1]], [1.0]) - ref))
        if lev == 2:
            ev = np.linalg.eigvals(P.lumped_preconditioned(m, Am))
            assert np.max(np.abs(ev - 0.5 * (1 + 4.0 / 80.0))) < 0.5
    order = math.log(err[0] / err[1]) / math.log(4.0)
    assert 0.85 < order < 1.15, (err, order)
    assert err[1] < 0.015 * abs(ref)


def test_matvec_rows_equal_dense_rows():
    """The row routine used at full size reproduces the dense P1 system."""
    v, t = synth.octa_sphere(2, 4.0)
    m = bem.make_mesh(v, t, 3)
    A_ = P.system_exterior(m, 4.0, 80.0, KAPPA)
    nv = len(v)
    x = np.random.default_rng(36).standard_normal(2 * nv)
    rows = np.array([0, 5, 33, nv - 1])
    got = P.matvec_rows(m, rows, x, 4.0, 80.0, KAPPA)
    ref = A_ @ x
    np.testing.assert_allclose(got[:, 0], ref[rows], rtol=1e-10, atol=1e-12)
    np.testing.assert_allclose(got[:, 1], ref[nv + rows], rtol=1e-10, atol=1e-12)


def test_energy_direct_equals_dense_energy():
    v, t = synth.octa_sphere(2, 4.0)
    m = bem.make_mesh(v, t, 3)
    x = np.random.default_rng(37).standard_normal(2 * len(v))
    qx, q = [[1.0, 1.0, 1.0], [-0.6, 0.3, -0.2]], [1.0, -0.5]
    assert P.energy_direct(m, x, qx, q) == pytest.approx(P.energy(m, x, qx, q), rel=1e-12)


def test_used_vertices_only_keeps_the_geometry():
    """The input helper that drops vertices no triangle uses (P1 unknowns
    live on vertices) renumbers triangles without moving them."""
    v, t = synth.octa_sphere(1, 2.0)
    extra = np.array([[9.0, 9.0, 9.0], [8.0, 8.0, 8.0]])
    v2 = np.concatenate([extra[:1], v, extra[1:]])
    t2 = t + 1
    v3, t3 = synth.used_vertices_only(v2, t2)
    assert len(v3) == len(v)
    np.testing.assert_array_equal(v3[t3], v2[t2])
