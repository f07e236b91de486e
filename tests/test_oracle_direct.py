"""Pins of the FP64 direct-sum oracle against closed forms, invariants and
finite differences (none of these re-types the oracle's formula)."""
import math

import numpy as np
import pytest

import synth
from oracle import direct as D

KAPPA = 0.125


@pytest.mark.parametrize("kernel", ["laplace", "yukawa"])
def test_single_source_closed_form(kernel):
    src = np.array([[0.5, -0.25, 1.0]])
    tgt = src + np.array([[0.0, 0.0, 3.0]])
    pot, grad = D.direct(tgt, src, np.array([2.0]), kernel, KAPPA)
    r = 3.0
    e = math.exp(-KAPPA * r) if kernel == "yukawa" else 1.0
    k = KAPPA if kernel == "yukawa" else 0.0
    assert pot[0] == pytest.approx(2.0 * e / (4 * math.pi * r), rel=1e-15)
    # d/dz of 2 e^{-k r}/(4 pi r) at r=3 along +z
    dz = -2.0 * (1 + k * r) * e / (4 * math.pi * r * r)
    assert grad[0, 2] == pytest.approx(dz, rel=1e-14)
    assert abs(grad[0, 0]) < 1e-18 and abs(grad[0, 1]) < 1e-18


@pytest.mark.parametrize("kernel", ["laplace", "yukawa"])
def test_gradient_is_derivative_of_potential(kernel):
    rng = np.random.default_rng(3)
    src = rng.uniform(-1, 1, (200, 3))
    q = rng.standard_normal(200)
    tgt = rng.uniform(2, 3, (5, 3))
    _, grad = D.direct(tgt, src, q, kernel, KAPPA)
    h = 1e-5
    for d in range(3):
        e = np.zeros(3)
        e[d] = h
        pp, _ = D.direct(tgt + e, src, q, kernel, KAPPA)
        pm, _ = D.direct(tgt - e, src, q, kernel, KAPPA)
        fd = (pp - pm) / (2 * h)
        np.testing.assert_allclose(grad[:, d], fd, rtol=1e-7, atol=1e-12)


@pytest.mark.parametrize("kernel,k", [("laplace", 0.0), ("yukawa", KAPPA), ("yukawa", 0.7)])
def test_helmholtz_operator_annihilates_potential(kernel, k):
    """(laplacian - kappa^2) phi = 0 away from the sources (7-point stencil)."""
    rng = np.random.default_rng(4)
    src = rng.uniform(-1, 1, (50, 3))
    q = rng.standard_normal(50)
    x0 = np.array([[3.0, 2.5, -2.0]])
    h = 2e-3
    p0, _ = D.direct(x0, src, q, kernel, k)
    lap = -6 * p0[0]
    for d in range(3):
        e = np.zeros(3)
        e[d] = h
        lap += D.direct(x0 + e, src, q, kernel, k)[0][0] + D.direct(x0 - e, src, q, kernel, k)[0][0]
    lap /= h * h
    assert abs(lap - k * k * p0[0]) < 1e-5 * (abs(p0[0]) + 1e-3)
    if kernel == "yukawa":
        assert abs(k * k * p0[0]) > 1e-4  # the kappa^2 term is really exercised


@pytest.mark.parametrize("kernel", ["laplace", "yukawa"])
def test_kernel_symmetry(kernel):
    x, _ = synth.unit_sphere_cloud(600, seed=5)
    rng = np.random.default_rng(5)
    a, b = rng.standard_normal(600), rng.standard_normal(600)
    ga, _ = D.direct(x, x, a, kernel, KAPPA)
    gb, _ = D.direct(x, x, b, kernel, KAPPA)
    assert float(a @ gb) == pytest.approx(float(b @ ga), rel=1e-12)


@pytest.mark.parametrize("kernel", ["laplace", "yukawa"])
def test_newton_third_law(kernel):
    x, q = synth.unit_sphere_cloud(700, seed=6)
    _, g = D.direct(x, x, q, kernel, KAPPA)
    tot = (q[:, None] * g).sum(axis=0)
    assert np.abs(tot).max() < 1e-11 * np.abs(q[:, None] * g).sum()


def test_kappa_zero_is_laplace():
    x, q = synth.unit_sphere_cloud(500, seed=7)
    pl, gl = D.direct(x, x, q, "laplace")
    py, gy = D.direct(x, x, q, "yukawa", 0.0)
    np.testing.assert_allclose(py, pl, rtol=1e-15, atol=0)
    np.testing.assert_allclose(gy, gl, rtol=1e-15, atol=0)


@pytest.mark.parametrize("kernel", ["laplace", "yukawa"])
def test_rigid_motion(kernel):
    x, q = synth.unit_sphere_cloud(400, seed=8)
    rng = np.random.default_rng(8)
    R = synth.random_rotation(rng)
    t = rng.standard_normal(3) * 10
    p0, g0 = D.direct(x, x, q, kernel, KAPPA)
    y = x @ R.T + t
    p1, g1 = D.direct(y, y, q, kernel, KAPPA)
    np.testing.assert_allclose(p1, p0, rtol=1e-11, atol=1e-12)
    np.testing.assert_allclose(g1, g0 @ R.T, rtol=1e-9, atol=1e-9)


def test_laplace_scaling():
    x, q = synth.unit_sphere_cloud(300, seed=9)
    p0, g0 = D.direct(x, x, q)
    p1, g1 = D.direct(2.5 * x, 2.5 * x, q)
    np.testing.assert_allclose(p1, p0 / 2.5, rtol=1e-12)
    np.testing.assert_allclose(g1, g0 / 2.5 ** 2, rtol=1e-11, atol=1e-13)


def test_coincident_points_excluded():
    x = np.array([[0.0, 0.0, 0.0], [0.0, 0.0, 0.0], [1.0, 0.0, 0.0]])
    q = np.array([1.0, 5.0, 2.0])
    p, g = D.direct(x, x, q)
    assert np.all(np.isfinite(p)) and np.all(np.isfinite(g))
    assert p[0] == pytest.approx(2.0 / (4 * math.pi))
    assert p[2] == pytest.approx(6.0 / (4 * math.pi))


@pytest.mark.parametrize("kernel", ["laplace", "yukawa"])
def test_uniform_shell(kernel):
    """Uniformly charged sphere of radius a, total charge Q: outside,
    Laplace Q/(4 pi R); Yukawa Q e^{-kR} sinh(ka)/(ka) / (4 pi R)."""
    n = 40000
    k = np.arange(n)
    z = 1 - (2 * k + 1) / n
    th = k * math.pi * (3 - math.sqrt(5))
    rho = np.sqrt(1 - z * z)
    a = 2.0
    x = a * np.stack([rho * np.cos(th), rho * np.sin(th), z], 1)
    Q = 3.0
    kap = 0.6
    tgt = np.array([[0.3, -0.2, 7.0]])
    R = float(np.linalg.norm(tgt))
    p, _ = D.direct(tgt, x, np.full(n, Q / n), kernel, kap)
    if kernel == "yukawa":
        ref = Q * math.exp(-kap * R) * math.sinh(kap * a) / (kap * a) / (4 * math.pi * R)
    else:
        ref = Q / (4 * math.pi * R)
    assert p[0] == pytest.approx(ref, rel=1e-6)


def test_numpy_and_c_versions_agree():
    x, q = synth.unit_sphere_cloud(300, seed=10)
    for kern in ("laplace", "yukawa"):
        p0, g0 = D.direct(x, x, q, kern, KAPPA)
        p1, g1 = D.direct_numpy(x, x, q, kern, KAPPA)
        np.testing.assert_allclose(p1, p0, rtol=1e-12)
        np.testing.assert_allclose(g1, g0, rtol=1e-10, atol=1e-12)
