"""Pins of the dense BEM oracle: quadrature exactness, the closed-form
triangle integrals against brute force, Gauss's theorem for the double
layer, the uniform-shell potentials for the single layer, and the Born and
Kirkwood solvation energies with first-order convergence."""
import math

import numpy as np
import pytest

import synth
from oracle import analytic as A
from oracle import bem

KAPPA = 0.125


def _mono_exact(a, b):
    # int over the unit right triangle of x^a y^b = a! b! / (a + b + 2)!
    return math.factorial(a) * math.factorial(b) / math.factorial(a + b + 2)


@pytest.mark.parametrize("npts,deg", [(3, 2), (6, 4)])
def test_regular_rules_exact_to_their_degree(npts, deg):
    bary, w = bem.regular_rule(npts)
    x, y = bary[:, 1], bary[:, 2]
    for a in range(deg + 1):
        for b in range(deg + 1 - a):
            assert 0.5 * np.sum(w * x ** a * y ** b) == pytest.approx(_mono_exact(a, b), rel=1e-12, abs=1e-15)
    # and not beyond (a sanity check that the test has teeth)
    assert abs(0.5 * np.sum(w * x ** (deg + 1)) - _mono_exact(deg + 1, 0)) > 1e-8


def test_collapsed_rule_exact():
    bary, w = bem.collapsed_rule(5)
    x, y = bary[:, 1], bary[:, 2]
    for a in range(8):
        for b in range(8 - a):
            assert 0.5 * np.sum(w * x ** a * y ** b) == pytest.approx(_mono_exact(a, b), rel=1e-12)


def _brute(x, tri, n, f):
    bary, w = bem.collapsed_rule(60)
    y = bary @ tri
    area = 0.5 * np.linalg.norm(np.cross(tri[1] - tri[0], tri[2] - tri[0]))
    return np.array([area * np.sum(w * f(xx, y)) for xx in x])


def test_closed_form_triangle_integrals_against_brute_force():
    tri = np.array([[0.0, 0.0, 0.0], [1.3, 0.1, 0.0], [0.2, 0.9, 0.1]])
    n = np.cross(tri[1] - tri[0], tri[2] - tri[0])
    n /= np.linalg.norm(n)
    rng = np.random.default_rng(31)
    x = tri.mean(axis=0) + rng.normal(0, 1.0, (12, 3)) + 1.5 * n
    pot = bem.tri_potential(x, tri, n)
    dlp = bem.tri_dlp(x, tri, n)
    bp = _brute(x, tri, n, lambda xx, y: 1.0 / np.linalg.norm(xx - y, axis=1))
    bd = _brute(x, tri, n, lambda xx, y: ((xx - y) @ n) / np.linalg.norm(xx - y, axis=1) ** 3)
    np.testing.assert_allclose(pot, bp, rtol=1e-9)
    np.testing.assert_allclose(dlp, bd, rtol=1e-7, atol=1e-12)


def test_solid_angles_of_a_closed_surface():
    """Gauss: sum over a closed outward-oriented surface of
    int n.(x-y)/|x-y|^3 is -4 pi inside and 0 outside."""
    v, t = synth.octa_sphere(2, 2.0)
    m = bem.make_mesh(v, t, 3)
    for x, ref in (([0.3, -0.2, 0.5], -4 * math.pi), ([0.0, 0.0, 3.5], 0.0)):
        tot = sum(bem.tri_dlp(np.array([x]), m.verts[m.tris[i]], m.normal[i])[0] for i in range(len(t)))
        assert tot == pytest.approx(ref, abs=1e-10)


def test_double_layer_of_a_constant_is_minus_half():
    """On a closed smooth surface the double layer of a constant density is
    -1/2 (the jump relation); tested on the sphere, row sums of K_L against
    -area/2."""
    v, t = synth.octa_sphere(3, 4.0)
    m = bem.make_mesh(v, t, 3)
    _, K = bem.operators(m, 0.0)
    ratio = K.sum(axis=1) / m.area
    assert np.abs(ratio + 0.5).max() < 0.02
    assert abs(ratio.mean() + 0.5) < 2e-3


@pytest.mark.parametrize("kappa", [0.0, 0.3])
def test_single_layer_of_a_constant_is_shell_potential(kappa):
    """Uniform unit density on a sphere of radius R, observed on the sphere:
    R (Laplace), (1 - exp(-2 kappa R)) / (2 kappa) (Yukawa)."""
    R = 4.0
    ref = R if kappa == 0 else (1 - math.exp(-2 * kappa * R)) / (2 * kappa)
    errs = []
    for lev in (2, 3):
        v, t = synth.octa_sphere(lev, R)
        m = bem.make_mesh(v, t, 3)
        V, _ = bem.operators(m, kappa)
        errs.append(abs((V.sum(axis=1) / m.area).mean() / ref - 1))
    # the flat-facet surface approaches the sphere at second order
    assert errs[1] < 1e-2 and errs[0] / errs[1] > 3.0, errs


def test_identical_pair_double_layer_vanishes():
    v, t = synth.octa_sphere(2, 4.0)
    m = bem.make_mesh(v, t, 3)
    V, K = bem.singular_entries(m, np.arange(5), np.arange(5), KAPPA)
    assert np.all(np.abs(K) < 1e-25) and np.all(V > 0)


def test_born_and_kirkwood_first_order_convergence():
    ref_b = A.born_energy(4.0, 1.0, 4.0, 80.0, KAPPA)
    ref_k = A.kirkwood_energy(4.0, [1, 1, 1], [1.0], 4.0, 80.0, KAPPA)
    eb, ek = [], []
    for lev in (2, 3):
        v, t = synth.octa_sphere(lev, 4.0)
        m = bem.make_mesh(v, t, 3)
        A_ = bem.system(m, 4.0, 80.0, KAPPA)
        for (qx, ref, store) in (([[0, 0, 0]], ref_b, eb), ([[1, 1, 1]], ref_k, ek)):
            b = bem.rhs(m, qx, [1.0], 4.0)
            x = np.linalg.solve(A_, b)
            store.append(abs(bem.energy(m, x, qx, [1.0]) - ref))
    # refinement by 4 in the number of elements divides the error by ~4
    for e in (eb, ek):
        order = math.log(e[0] / e[1]) / math.log(4.0)
        assert 0.85 < order < 1.15, (e, order)
    assert ek[1] / abs(ref_k) < 0.015


def test_matvec_rows_equal_dense_rows():
    """The row routine used for large meshes reproduces the dense operator."""
    v, t = synth.octa_sphere(2, 4.0)
    m = bem.make_mesh(v, t, 3)
    A_ = bem.system(m, 4.0, 80.0, KAPPA)
    x = np.random.default_rng(33).standard_normal(2 * len(t))
    rows = np.array([0, 5, 17, 100])
    got = bem.matvec_rows(m, rows, x, 4.0, 80.0, KAPPA)
    ref = A_ @ x
    np.testing.assert_allclose(got[:, 0], ref[rows], rtol=1e-11, atol=1e-13)
    np.testing.assert_allclose(got[:, 1], ref[len(t) + rows], rtol=1e-11, atol=1e-13)


def test_reaction_potential_direct_equals_dense():
    v, t = synth.octa_sphere(2, 4.0)
    m = bem.make_mesh(v, t, 3)
    rng = np.random.default_rng(34)
    x = rng.standard_normal(2 * len(t))
    qx = rng.uniform(-2.0, 2.0, (7, 3))
    np.testing.assert_allclose(bem.reaction_potential_direct(m, x, qx), bem.reaction_potential(m, x, qx),
                               rtol=1e-12, atol=1e-13)


# ---- derivative (Juffer) formulation -------------------------------------
def _h(r, kappa):
    return (math.exp(-kappa * r) - 1.0) / (4.0 * math.pi * r)


def test_hyper_diff_kernel_against_finite_differences():
    """-d2/(dn_x dn_y) of g_Y - g_L, against central differences of the
    kernel along both normals."""
    rng = np.random.default_rng(151)
    for _ in range(6):
        x, y = rng.standard_normal(3), 0.4 * rng.standard_normal(3)
        nx, ny = rng.standard_normal(3), rng.standard_normal(3)
        nx /= np.linalg.norm(nx)
        ny /= np.linalg.norm(ny)
        e = 1e-4
        H = lambda a, b: _h(float(np.linalg.norm(a - b)), KAPPA)  # noqa: E731
        fd = -(H(x + e * nx, y + e * ny) - H(x + e * nx, y - e * ny) - H(x - e * nx, y + e * ny)
               + H(x - e * nx, y - e * ny)) / (4 * e * e)
        assert abs(bem.hyper_diff_kernel(x - y, nx, ny, KAPPA) - fd) < 2e-5 * abs(fd) + 5e-10


def test_h_remainder_series_matches_closed_form():
    r = np.array([0.3, 0.39, 0.41, 1.0, 3.0])
    _, A_, _ = bem._h_derivs(r, KAPPA)
    hp = np.array([(1 - (1 + KAPPA * rr) * math.exp(-KAPPA * rr)) / (4 * math.pi * rr * rr) for rr in r])
    ref = hp / r - KAPPA ** 2 / (8 * math.pi * r)
    np.testing.assert_allclose(A_, ref, rtol=1e-6)
    # the bounded remainder tends to -kappa^3 / (12 pi)
    assert abs(bem._h_derivs(np.array([1e-6]), KAPPA)[1][0] + KAPPA ** 3 / (12 * math.pi)) < 1e-10


def test_hyper_diff_singular_rule_converges():
    v, t = synth.octa_sphere(3, 4.0)
    m = bem.make_mesh(v, t, 3)
    sp = np.array(bem.singular_pairs(m))[:60]
    a = bem.hyper_diff_singular(m, sp[:, 0], sp[:, 1], KAPPA, 8, 4)
    b = bem.hyper_diff_singular(m, sp[:, 0], sp[:, 1], KAPPA, 16, 12)
    assert np.max(np.abs(a - b) / np.abs(b)) < 2e-3


def test_adjoint_double_layer_is_the_transpose():
    """K'[s,t] = int_Ts int_Tt dg/dn_x: for a few regular pairs, from the
    definition, against K[t,s] of the dense operator."""
    v, t = synth.octa_sphere(2, 4.0)
    m = bem.make_mesh(v, t, 3)
    _, K = bem.operators(m, KAPPA)
    for s_, t_ in ((0, 40), (7, 90), (33, 2)):
        x, y = m.qpts[s_], m.qpts[t_]
        d = x[:, None, :] - y[None, :, :]
        r = np.linalg.norm(d, axis=2)
        dgdnx = -(d @ m.normal[s_]) * (1 + KAPPA * r) * np.exp(-KAPPA * r) / (4 * math.pi * r ** 3)
        kp = float(np.sum(m.qw[s_][:, None] * m.qw[t_][None, :] * dgdnx))
        assert abs(kp - K[t_, s_]) < 1e-12 * abs(kp) + 1e-18


def test_derivative_formulation_converges_and_stays_conditioned():
    """Kirkwood sphere: the derivative formulation's energy converges at
    order 1 like the direct one, and its condition number stays flat under
    refinement while the direct formulation's grows (Methods: the direct
    form's condition number grows with the number of elements)."""
    ref = A.kirkwood_energy(4.0, [1, 1, 1], [1.0], 4.0, 80.0, KAPPA)
    err, cond_d, cond_0 = [], [], []
    for lev in (2, 3):
        v, t = synth.octa_sphere(lev, 4.0)
        m = bem.make_mesh(v, t, 3)
        x, Ad, _ = bem.solve_derivative(m, [[1, 1, 1]], [1.0])
        err.append(abs(bem.energy(m, x, [[1, 1, 1]], [1.0]) - ref))
        cond_d.append(np.linalg.cond(Ad))
        cond_0.append(np.linalg.cond(bem.system(m, 4.0, 80.0, KAPPA)))
    order = math.log(err[0] / err[1]) / math.log(4.0)
    assert 0.85 < order < 1.15, (err, order)
    assert cond_d[1] / cond_d[0] < 1.1 and cond_0[1] / cond_0[0] > 1.5


# ---- exterior derivative formulation (eq:lu) ------------------------------
def test_exterior_formulation_meets_the_interface_conditions():
    """eq:lu is solved for the solvent-side unknowns; mapped through the
    interface conditions (continuous potential, eps1 dphi_1/dn = eps2
    dphi_2/dn) its solution must be the Juffer solution of eq:juffer."""
    v, t = synth.octa_sphere(2, 4.0)
    m = bem.make_mesh(v, t, 3)
    qx, q = [[1.0, 1.0, 1.0], [-0.7, 0.2, 0.4]], [1.0, -0.5]
    xe, _, _ = bem.solve_exterior(m, qx, q)
    xj, _, _ = bem.solve_derivative(m, qx, q)
    np.testing.assert_allclose(bem.interior_unknowns(xe, 4.0, 80.0), xj, rtol=1e-10, atol=1e-12 * np.abs(xj).max())


def test_exterior_formulation_kirkwood_convergence():
    ref = A.kirkwood_energy(4.0, [1, 1, 1], [1.0], 4.0, 80.0, KAPPA)
    err = []
    for lev in (2, 3):
        v, t = synth.octa_sphere(lev, 4.0)
        m = bem.make_mesh(v, t, 3)
        xe, _, _ = bem.solve_exterior(m, [[1, 1, 1]], [1.0])
        err.append(abs(bem.energy(m, bem.interior_unknowns(xe, 4.0, 80.0), [[1, 1, 1]], [1.0]) - ref))
    order = math.log(err[0] / err[1]) / math.log(4.0)
    assert 0.85 < order < 1.15, (err, order)


def _gmres_iterations(Am, b, tol=1e-8, maxit=200):
    """Iterations of full GMRES (no restart) to a relative residual tol."""
    n = len(b)
    beta = np.linalg.norm(b)
    V = np.zeros((n, maxit + 1))
    H = np.zeros((maxit + 1, maxit))
    V[:, 0] = b / beta
    for j in range(maxit):
        w = Am @ V[:, j]
        for _ in range(2):
            h = V[:, :j + 1].T @ w
            w -= V[:, :j + 1] @ h
            H[:j + 1, j] += h
        H[j + 1, j] = np.linalg.norm(w)
        V[:, j + 1] = w / H[j + 1, j]
        e1 = np.zeros(j + 2)
        e1[0] = beta
        y = np.linalg.lstsq(H[:j + 2, :j + 1], e1, rcond=None)[0]
        if np.linalg.norm(H[:j + 2, :j + 1] @ y - e1) <= tol * beta:
            return j + 1
    return maxit


def test_mass_preconditioned_spectra_and_iterations():
    """Under mass-matrix preconditioning the interior (Juffer) operator's
    eigenvalues gather at (1 + eps2/eps1)/2 and (1 + eps1/eps2)/2, the
    exterior operator's at (1 + eps1/eps2)/2 alone, and GMRES on the exterior
    form needs about half the iterations (Results: the two derivative
    variants and their eigenvalues)."""
    v, t = synth.octa_sphere(2, 4.0)
    m = bem.make_mesh(v, t, 3)
    lo, hi = 0.5 * (1 + 4.0 / 80.0), 0.5 * (1 + 80.0 / 4.0)
    Aj = bem.mass_preconditioned(m, bem.system_derivative(m, 4.0, 80.0, KAPPA))
    Ae = bem.mass_preconditioned(m, bem.system_exterior(m, 4.0, 80.0, KAPPA))
    ej, ee = np.linalg.eigvals(Aj), np.linalg.eigvals(Ae)
    assert np.max(np.abs(ee - lo)) < 0.5
    assert np.mean(np.abs(ej - lo) < 0.5) > 0.45 and np.mean(np.abs(ej - hi) < 2.0) > 0.45
    d = np.concatenate([m.area, m.area])
    qx, q = [[1.0, 1.0, 1.0]], [1.0]
    it_j = _gmres_iterations(Aj, bem.rhs_derivative(m, qx, q, 4.0) / d)
    it_e = _gmres_iterations(Ae, bem.rhs_exterior(m, qx, q, 80.0) / d)
    assert it_e <= 0.6 * it_j, (it_e, it_j)


@pytest.mark.parametrize("formulation", ["interior", "exterior"])
def test_derivative_matvec_rows_equal_dense_rows(formulation):
    """The row routine used at full size reproduces the dense derivative
    systems (eq:juffer and eq:lu)."""
    v, t = synth.octa_sphere(2, 4.0)
    m = bem.make_mesh(v, t, 3)
    A_ = (bem.system_derivative if formulation == "interior" else bem.system_exterior)(m, 4.0, 80.0, KAPPA)
    x = np.random.default_rng(35).standard_normal(2 * len(t))
    rows = np.array([0, 9, 64, 127])
    got = bem.matvec_rows_derivative(m, rows, x, 4.0, 80.0, KAPPA, formulation=formulation)
    ref = A_ @ x
    np.testing.assert_allclose(got[:, 0], ref[rows], rtol=1e-10, atol=1e-12)
    np.testing.assert_allclose(got[:, 1], ref[len(t) + rows], rtol=1e-10, atol=1e-12)
