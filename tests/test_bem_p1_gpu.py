"""GPU parity of the exterior derivative formulation on P1 elements (eq:lu
with continuous piecewise-linear unknowns per vertex) against the dense FP64
P1 oracle: matvec, right-hand side, lumped-mass preconditioner, GMRES
solution and energy, and the argument checks of the P1 path."""
import numpy as np
import pytest

import synth
from oracle import bem as B
from oracle import bem_p1 as P
from tests.gpu_util import require_gpu

pytestmark = pytest.mark.gpu
KAPPA = 0.125


def _rel(a, b):
    return float(np.linalg.norm(np.asarray(a) - np.asarray(b)) / np.linalg.norm(b))


def _op(v, t, precision, p=8, ncrit=64, quad=3):
    require_gpu()
    from paper_2103_01048_amd import BEMOperator
    return BEMOperator(v, t, quad_pts=quad, eps_in=4.0, eps_out=80.0, kappa=KAPPA, p=p, ncrit=ncrit,
                       precision=precision, formulation="exterior_p1")


@pytest.fixture(scope="module")
def sphere512():
    v, t = synth.octa_sphere(3, 4.0)
    m = B.make_mesh(v, t, 3)
    return v, t, m, P.system_exterior(m, 4.0, 80.0, KAPPA)


@pytest.mark.parametrize("precision,tol", [("fp64", 1e-6), ("fp32", 1e-4), ("bf16x3", 1e-4)])
def test_p1_matvec_matches_dense_oracle(sphere512, precision, tol):
    torch = require_gpu()
    v, t, m, A_ = sphere512
    op = _op(v, t, precision)
    info = op.info()
    assert info["formulation"] == 3 and info["n_unknowns"] == len(v) and info["preconditioner"] == 1
    rng = np.random.default_rng(171)
    for _ in range(2):
        x = rng.standard_normal(2 * len(v))
        y = op.matvec(torch.tensor(x, device="cuda")).cpu().numpy()
        e = _rel(y, A_ @ x)
        print(f"[P1 matvec {precision}] rel {e:.2e}", flush=True)
        assert e < tol


@pytest.mark.parametrize("quad", [3, 6])
def test_p1_matvec_sphere_union_mesh(quad):
    """An open sphere-union surface (buried triangles dropped) over several
    leaves, both regular rules."""
    torch = require_gpu()
    su = synth.sphere_union_spheres(12, seed=172, box=8.0)
    v, t = synth.used_vertices_only(*synth.sphere_union_mesh(su, 900, seed=172, gap=0.5))
    m = B.make_mesh(v, t, quad)
    A_ = P.system_exterior(m, 4.0, 80.0, KAPPA)
    x = np.random.default_rng(172).standard_normal(2 * len(v))
    y = _op(v, t, "fp64", ncrit=48, quad=quad).matvec(torch.tensor(x, device="cuda")).cpu().numpy()
    e = _rel(y, A_ @ x)
    print(f"[P1 matvec sphere union, {quad} points] rel {e:.2e}", flush=True)
    assert e < 1e-6


def test_p1_rhs_and_preconditioner(sphere512):
    torch = require_gpu()
    v, t, m, _ = sphere512
    op = _op(v, t, "fp64")
    qx = np.array([[1.0, 1.0, 1.0], [-0.5, 0.2, 0.3]])
    q = np.array([1.0, -0.4])
    b = op.rhs(qx, q).cpu().numpy()
    np.testing.assert_allclose(b, P.rhs_exterior(m, qx, q, 80.0), rtol=1e-12, atol=1e-15)
    x = np.random.default_rng(173).standard_normal(2 * len(v))
    z = op.precondition(torch.tensor(x, device="cuda")).cpu().numpy()
    np.testing.assert_allclose(z, x / np.concatenate([P.lumped_mass(m)] * 2), rtol=1e-14)
    with pytest.raises(RuntimeError):
        op.set_preconditioner("block")
    with pytest.raises(ValueError):
        op.matvec(torch.zeros(2 * len(t), dtype=torch.float64, device="cuda"))


def test_p1_gmres_solution_and_energy(sphere512):
    require_gpu()
    from paper_2103_01048_amd import gmres
    v, t, m, A_ = sphere512
    qx, q = [[1.0, 1.0, 1.0], [-0.6, 0.3, -0.2]], [1.0, -0.5]
    x_lu = np.linalg.solve(A_, P.rhs_exterior(m, qx, q, 80.0))
    e_lu = P.energy(m, x_lu, qx, q)
    op = _op(v, t, "fp64", p=10)
    b = op.rhs(qx, q)
    x, it, hist, rc = gmres(op, b, tol=1e-10, maxiter=200)
    print(f"[P1 gmres fp64] {it} iterations, rc {rc}", flush=True)
    assert rc == 0 and it < 40
    xs = x.cpu().numpy()
    assert _rel(xs, x_lu) < 1e-7
    assert op.energy(x, qx, q) == pytest.approx(e_lu, rel=1e-7)
    # the energy of the oracle's own solution: the quadrature sum alone
    import torch
    assert op.energy(torch.tensor(x_lu, device="cuda"), qx, q) == pytest.approx(e_lu, rel=1e-12)
    # bf16x3 inner solves refined against the FP64 operator
    lo = _op(v, t, "bf16x3")
    x2, it2, _, rc2 = gmres(lo, b, tol=1e-8, maxiter=200, refine=op)
    print(f"[P1 gmres bf16x3 + refinement] {it2} iterations, rc {rc2}", flush=True)
    assert rc2 == 0
    assert _rel(x2.cpu().numpy(), x_lu) < 1e-6


def test_p1_rejects_a_vertex_on_no_triangle():
    require_gpu()
    v, t = synth.octa_sphere(1, 2.0)
    v = np.concatenate([v, [[9.0, 9.0, 9.0]]])
    with pytest.raises(RuntimeError):
        _op(v, t, "fp64")


def test_p1_no_charges_and_determinism(sphere512):
    """No charges: a zero right-hand side and zero energy; two matvecs of the
    same vector are bitwise equal (fixed-order sums per vertex)."""
    torch = require_gpu()
    v, t, m, _ = sphere512
    op = _op(v, t, "bf16x3")
    b = op.rhs(np.zeros((0, 3)), np.zeros(0)).cpu().numpy()
    assert b.shape == (2 * len(v),) and not b.any()
    x = torch.tensor(np.random.default_rng(174).standard_normal(2 * len(v)), device="cuda")
    assert op.energy(x, np.zeros((0, 3)), np.zeros(0)) == 0.0
    assert torch.equal(op.matvec(x), op.matvec(x))
