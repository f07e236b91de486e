"""GPU parity of the derivative (Juffer) formulation (eq:juffer, P0
Galerkin) against the dense FP64 oracle: matvec, right-hand side, GMRES
solution and energy; Kirkwood convergence and its iteration counts against
the direct formulation on the same meshes."""
import math

import numpy as np
import pytest

import synth
from oracle import analytic as A
from oracle import bem as B
from tests.gpu_util import require_gpu

pytestmark = pytest.mark.gpu
KAPPA = 0.125


def _rel(a, b):
    return float(np.linalg.norm(np.asarray(a) - np.asarray(b)) / np.linalg.norm(b))


def _op(v, t, precision, p=8, ncrit=64, quad=3, formulation="derivative"):
    require_gpu()
    from paper_2103_01048_amd import BEMOperator
    return BEMOperator(v, t, quad_pts=quad, eps_in=4.0, eps_out=80.0, kappa=KAPPA, p=p, ncrit=ncrit,
                       precision=precision, formulation=formulation)


@pytest.fixture(scope="module")
def sphere512():
    v, t = synth.octa_sphere(3, 4.0)
    m = B.make_mesh(v, t, 3)
    return v, t, m, B.system_derivative(m, 4.0, 80.0, KAPPA)


@pytest.mark.parametrize("precision,tol", [("fp64", 1e-6), ("fp32", 1e-4), ("bf16x3", 1e-4)])
def test_derivative_matvec_matches_dense_oracle(sphere512, precision, tol):
    torch = require_gpu()
    v, t, m, A_ = sphere512
    op = _op(v, t, precision)
    assert op.info()["formulation"] == 1
    rng = np.random.default_rng(161)
    for _ in range(2):
        x = rng.standard_normal(2 * len(t))
        y = op.matvec(torch.tensor(x, device="cuda")).cpu().numpy()
        e = _rel(y, A_ @ x)
        print(f"[derivative matvec {precision}] rel {e:.2e}", flush=True)
        assert e < tol


def test_derivative_matvec_sphere_union_mesh():
    torch = require_gpu()
    su = synth.sphere_union_spheres(12, seed=162, box=8.0)
    v, t = synth.sphere_union_mesh(su, 1200, seed=162, gap=0.5)
    m = B.make_mesh(v, t, 3)
    A_ = B.system_derivative(m, 4.0, 80.0, KAPPA)
    x = np.random.default_rng(162).standard_normal(2 * len(t))
    y = _op(v, t, "fp64", ncrit=48).matvec(torch.tensor(x, device="cuda")).cpu().numpy()
    assert _rel(y, A_ @ x) < 1e-6


def test_derivative_rhs_matches_oracle(sphere512):
    require_gpu()
    v, t, m, _ = sphere512
    op = _op(v, t, "fp64")
    qx = np.array([[1.0, 1.0, 1.0], [-0.5, 0.2, 0.3]])
    q = np.array([1.0, -0.4])
    b = op.rhs(qx, q).cpu().numpy()
    np.testing.assert_allclose(b, B.rhs_derivative(m, qx, q, 4.0), rtol=1e-12, atol=1e-15)


def test_derivative_gmres_solution_and_energy(sphere512):
    require_gpu()
    from paper_2103_01048_amd import gmres
    v, t, m, A_ = sphere512
    qx, q = [[1.0, 1.0, 1.0]], [1.0]
    x_lu = np.linalg.solve(A_, B.rhs_derivative(m, qx, q, 4.0))
    e_lu = B.energy(m, x_lu, qx, q)
    op = _op(v, t, "fp64")
    b = op.rhs(qx, q)
    x, it, hist, rc = gmres(op, b, tol=1e-10, maxiter=300)
    assert rc == 0 and 0 < it < 300
    assert _rel(x.cpu().numpy(), x_lu) < 1e-5
    e = op.energy(x, qx, q)
    print(f"[derivative energy] gpu {e:.8f} oracle {e_lu:.8f} iters {it}", flush=True)
    assert e == pytest.approx(e_lu, rel=1e-6)


def test_derivative_kirkwood_convergence_and_iterations():
    """Order-1 convergence to Kirkwood's energy, in fewer GMRES iterations
    than the direct formulation, whose count grows with refinement."""
    require_gpu()
    from paper_2103_01048_amd import gmres
    ref = A.kirkwood_energy(4.0, [1, 1, 1], [1.0], 4.0, 80.0, KAPPA)
    errs, its_d, its_0 = [], [], []
    for lev in (3, 4, 5):
        v, t = synth.octa_sphere(lev, 4.0)
        for form, store in (("derivative", its_d), ("direct", its_0)):
            op = _op(v, t, "fp64", ncrit=64, quad=6, formulation=form)
            b = op.rhs([[1.0, 1.0, 1.0]], [1.0])
            x, it, _, rc = gmres(op, b, tol=1e-8, maxiter=500)
            assert rc == 0
            store.append(it)
            if form == "derivative":
                e = op.energy(x, [[1.0, 1.0, 1.0]], [1.0])
                errs.append(abs(e - ref))
                print(f"[derivative kirkwood] T={len(t)} dG={e:.6f} ref={ref:.6f} iters={it}", flush=True)
    print(f"[iterations] derivative {its_d} direct {its_0}", flush=True)
    for a, b in zip(errs, errs[1:]):
        order = math.log(a / b) / math.log(4.0)
        assert 0.85 < order < 1.15, errs
    assert all(d < o for d, o in zip(its_d, its_0))


# ---- exterior derivative formulation (eq:lu) and the mass preconditioner ----
@pytest.fixture(scope="module")
def sphere512_ext():
    v, t = synth.octa_sphere(3, 4.0)
    m = B.make_mesh(v, t, 3)
    return v, t, m, B.system_exterior(m, 4.0, 80.0, KAPPA)


@pytest.mark.parametrize("precision,tol", [("fp64", 1e-6), ("fp32", 1e-4), ("bf16x3", 1e-4)])
def test_exterior_matvec_matches_dense_oracle(sphere512_ext, precision, tol):
    torch = require_gpu()
    v, t, m, A_ = sphere512_ext
    op = _op(v, t, precision, formulation="exterior")
    assert op.info()["formulation"] == 2
    x = np.random.default_rng(171).standard_normal(2 * len(t))
    y = op.matvec(torch.tensor(x, device="cuda")).cpu().numpy()
    e = _rel(y, A_ @ x)
    print(f"[exterior matvec {precision}] rel {e:.2e}", flush=True)
    assert e < tol


def test_exterior_rhs_gmres_and_energy(sphere512_ext):
    require_gpu()
    from paper_2103_01048_amd import gmres
    v, t, m, A_ = sphere512_ext
    qx, q = np.array([[1.0, 1.0, 1.0], [-0.5, 0.2, 0.3]]), np.array([1.0, -0.4])
    op = _op(v, t, "fp64", formulation="exterior")
    b = op.rhs(qx, q)
    b_ref = B.rhs_exterior(m, qx, q, 80.0)
    np.testing.assert_allclose(b.cpu().numpy(), b_ref, rtol=1e-12, atol=1e-15)
    x_lu = np.linalg.solve(A_, b_ref)
    e_lu = B.energy(m, B.interior_unknowns(x_lu, 4.0, 80.0), qx, q)
    for pre in ("block", "mass"):
        op.set_preconditioner(pre)
        x, it, _, rc = gmres(op, b, tol=1e-10, maxiter=300) if pre == "block" else op.solve(b, tol=1e-10, maxiter=300)
        assert rc == 0 and 0 < it < 300
        assert _rel(x.cpu().numpy(), x_lu) < 1e-5
        e = op.energy(x, qx, q)
        print(f"[exterior energy {pre}] gpu {e:.8f} oracle {e_lu:.8f} iters {it}", flush=True)
        assert e == pytest.approx(e_lu, rel=1e-6)


def test_mass_preconditioner_is_the_inverse_area():
    torch = require_gpu()
    v, t = synth.octa_sphere(2, 4.0)
    m = B.make_mesh(v, t, 3)
    op = _op(v, t, "fp64", formulation="exterior")
    op.set_preconditioner("mass")
    assert op.info()["preconditioner"] == 1
    x = np.random.default_rng(172).standard_normal(2 * len(t))
    y = op.precondition(torch.tensor(x, device="cuda")).cpu().numpy()
    np.testing.assert_allclose(y, x / np.concatenate([m.area, m.area]), rtol=1e-14)


def test_exterior_converges_in_fewer_iterations_under_mass_preconditioning():
    """Kirkwood sphere with the mass preconditioner: the exterior form
    converges at order 1 to Kirkwood's energy in about half the GMRES
    iterations of the interior (Juffer) form (Results: the two derivative
    variants)."""
    require_gpu()
    from paper_2103_01048_amd import gmres
    ref = A.kirkwood_energy(4.0, [1, 1, 1], [1.0], 4.0, 80.0, KAPPA)
    errs, its = [], {"derivative": [], "exterior": []}
    for lev in (3, 4, 5):
        v, t = synth.octa_sphere(lev, 4.0)
        for form in ("derivative", "exterior"):
            op = _op(v, t, "fp64", ncrit=64, quad=6, formulation=form)
            op.set_preconditioner("mass")
            b = op.rhs([[1.0, 1.0, 1.0]], [1.0])
            x, it, _, rc = gmres(op, b, tol=1e-8, maxiter=500)
            assert rc == 0
            its[form].append(it)
            e = op.energy(x, [[1.0, 1.0, 1.0]], [1.0])
            if form == "exterior":
                errs.append(abs(e - ref))
            print(f"[mass-preconditioned {form}] T={len(t)} dG={e:.6f} ref={ref:.6f} iters={it}", flush=True)
    print(f"[iterations, mass preconditioner] {its}", flush=True)
    for a, b in zip(errs, errs[1:]):
        order = math.log(a / b) / math.log(4.0)
        assert 0.85 < order < 1.15, errs
    assert all(e <= 0.6 * d for e, d in zip(its["exterior"], its["derivative"])), its


def test_exterior_refinement_from_the_bf16x3_operator(sphere512_ext):
    """GMRES on the bf16x3 exterior operator with FP64 residuals (iterative
    refinement against the FP64 operator) reaches the dense solution."""
    require_gpu()
    from paper_2103_01048_amd import gmres
    v, t, m, A_ = sphere512_ext
    qx, q = [[1.0, 1.0, 1.0]], [1.0]
    op = _op(v, t, "bf16x3", formulation="exterior")
    ref = _op(v, t, "fp64", formulation="exterior")
    op.set_preconditioner("mass")
    b = ref.rhs(qx, q)
    x, it, _, rc = gmres(op, b, tol=1e-9, maxiter=300, refine=ref, inner_tol=1e-3)
    assert rc == 0
    x_lu = np.linalg.solve(A_, B.rhs_exterior(m, qx, q, 80.0))
    e = _rel(x.cpu().numpy(), x_lu)
    print(f"[exterior refinement] iterations {it} rel {e:.2e}", flush=True)
    assert e < 1e-6


def test_set_preconditioner_rejects_unknown_kind():
    require_gpu()
    from paper_2103_01048_amd import _lib
    from paper_2103_01048_amd._lib import lib
    v, t = synth.octa_sphere(2, 4.0)
    op = _op(v, t, "fp32", formulation="exterior")
    assert lib().bem_set_preconditioner(op._h, 7, None) == _lib.FMM_EINVAL
    assert "preconditioner" in lib().fmm_last_error().decode()
    with pytest.raises(ValueError):
        op.set_preconditioner("jacobi")
    assert op.info()["preconditioner"] == 0
