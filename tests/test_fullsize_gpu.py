"""GPU parity at the workloads' full sizes, in the launch configurations the
benchmark times, on sampled outputs that the FP64 oracle computes one by one
(single rows of the N-body sums and of the boundary-element matrix, finite
differences of the exact pair energy), plus properties that hold at any size
(GMRES residual of the FP64 operator).

Workloads (all seeded, synthetic sphere-union surfaces):
* 393,216 points (131,072 triangles x 3) on 200 spheres, Laplace and Yukawa
  kappa = 0.125, p = 8, each ncrit of the benchmark's sweep;
* the same surface at 1,000,002 points (500 spheres) for the adjoint;
* 64 molecules of 5k-60k points in one batched plan;
* 2M triangles x 3 points on 1,000 spheres for the boundary-element solve
  with 20,000 charges (caps of intersecting spheres stop half an edge
  length short of each other: triangles that cross near an intersection
  curve make GMRES stagnate);
* 30M points (10M triangles x 3) on a 30,000-sphere shell of radius 200 A,
  p = 10.

Tolerances: 1e-4 relative L2 over the sampled rows for every single-precision
path (the accuracy target of the mixed-precision evaluation) and 1e-6 for
FP64 at p = 8; position gradients of the FP32 adjoint 1e-3 (the FMM's
gradient is one order less accurate than its potential)."""
import math

import numpy as np
import pytest

import synth
from oracle import bem as B
from oracle import direct as D
from tests.gpu_util import require_gpu

pytestmark = [pytest.mark.gpu, pytest.mark.fullsize]
KAPPA = 0.125


def _rel(a, b):
    a, b = np.asarray(a, dtype=np.float64), np.asarray(b, dtype=np.float64)
    return float(np.linalg.norm(a - b) / np.linalg.norm(b))


def _say(msg):
    print(msg, flush=True)


def _check_rows(plan, torch, x, q, rows, kernel, tol, tag):
    pot, grad = plan.eval(torch.tensor(q, device="cuda"))
    torch.cuda.synchronize()
    phi, g = D.direct(x[rows], x, q, kernel, KAPPA if kernel == "yukawa" else 0.0)
    ep = _rel(pot.cpu().numpy()[rows], phi)
    eg = _rel(grad.cpu().numpy()[rows], g)
    _say(f"[{tag}] pot {ep:.2e} grad {eg:.2e}")
    assert ep < tol and eg < tol


@pytest.fixture(scope="module")
def surface393k():
    _say("[fullsize] building the 393,216-point surface")
    return synth.surface_cloud(200, 131072, seed=1, box=40.0)


@pytest.mark.parametrize("ncrit", [64, 128, 256])
@pytest.mark.parametrize("kernel", ["laplace", "yukawa"])
def test_surface393k_bf16x3_every_ncrit(surface393k, kernel, ncrit):
    torch = require_gpu()
    from paper_2103_01048_amd import FMMPlan
    x, q = surface393k
    plan = FMMPlan(torch.tensor(x, device="cuda"), kernel=kernel, kappa=KAPPA, p=8, ncrit=ncrit,
                   precision="bf16x3")
    rows = np.random.default_rng(71).choice(len(x), 2048, replace=False)
    _check_rows(plan, torch, x, q, rows, kernel, 1e-4, f"393k {kernel} bf16x3 ncrit {ncrit}")


@pytest.mark.parametrize("precision,tol,ncrit", [("bf16x3", 1e-4, nc) for nc in (64, 96, 128, 192, 256)]
                         + [("fp32", 1e-4, 128), ("fp64", 1e-6, 128)])
def test_surface393k_pair(surface393k, precision, tol, ncrit):
    """The benchmark's step: one fmm_eval_pair of a Laplace and a Yukawa
    plan (p = 8, every ncrit of the benchmark's sweep) against the direct
    sums on sampled rows."""
    torch = require_gpu()
    from paper_2103_01048_amd import FMMPlan, eval_pair
    x, q = surface393k
    xt = torch.tensor(x, device="cuda")
    plans = [FMMPlan(xt, kernel=k, kappa=KAPPA, p=8, ncrit=ncrit, precision=precision) for k in ("laplace", "yukawa")]
    outs = eval_pair(plans[0], plans[1], torch.tensor(q, device="cuda"))
    torch.cuda.synchronize()
    rows = np.random.default_rng(74).choice(len(x), 2048, replace=False)
    for kernel, (pot, grad) in zip(("laplace", "yukawa"), outs):
        phi, g = D.direct(x[rows], x, q, kernel, KAPPA if kernel == "yukawa" else 0.0)
        ep = _rel(pot.cpu().numpy()[rows], phi)
        eg = _rel(grad.cpu().numpy()[rows], g)
        _say(f"[393k pair {precision} ncrit {ncrit} {kernel}] pot {ep:.2e} grad {eg:.2e}")
        assert ep < tol and eg < tol


@pytest.mark.parametrize("precision,tol,tuning", [
    ("bf16x3", 1e-4, {"work_cap_div": 32768}),
    ("bf16x3", 1e-4, {"work_cap_div": 32768, "m2l_factored": 1}),
    ("fp64", 1e-6, {"work_cap_div": 32768, "m2l_factored": 1}),
])
def test_surface393k_pair_tuned_and_factored(surface393k, precision, tol, tuning):
    """The benchmark's step in the autotuned configuration (ncrit 160, leaf
    items cut at total/32768) and with the per-offset factored M2L, against
    the direct sums on sampled rows."""
    torch = require_gpu()
    from paper_2103_01048_amd import FMMPlan, autotune as at, eval_pair
    x, q = surface393k
    xt = torch.tensor(x, device="cuda")
    with at.tuning(**tuning):
        plans = [FMMPlan(xt, kernel=k, kappa=KAPPA, p=8, ncrit=160, precision=precision)
                 for k in ("laplace", "yukawa")]
    outs = eval_pair(plans[0], plans[1], torch.tensor(q, device="cuda"))
    torch.cuda.synchronize()
    rows = np.random.default_rng(75).choice(len(x), 2048, replace=False)
    for kernel, (pot, grad) in zip(("laplace", "yukawa"), outs):
        phi, g = D.direct(x[rows], x, q, kernel, KAPPA if kernel == "yukawa" else 0.0)
        ep = _rel(pot.cpu().numpy()[rows], phi)
        eg = _rel(grad.cpu().numpy()[rows], g)
        _say(f"[393k pair {precision} {tuning} {kernel}] pot {ep:.2e} grad {eg:.2e}")
        assert ep < tol and eg < tol


def _shipped(at, n, p, precision, device):
    key = at.cache_key(n, p, precision, device)
    entry = at.shipped_table().get(key)
    if entry is None:
        pytest.skip(f"no shipped tuning entry for {key}")
    return entry


def _pair_rows(plans, torch, x, q, rows, tol, tag):
    from paper_2103_01048_amd import eval_pair
    dt = torch.float64 if plans[0].precision == "fp64" else torch.float32
    outs = eval_pair(plans[0], plans[1], torch.tensor(q, device="cuda", dtype=dt))
    torch.cuda.synchronize()
    for kernel, (pot, grad) in zip(("laplace", "yukawa"), outs):
        phi, g = D.direct(x[rows], x, q, kernel, KAPPA if kernel == "yukawa" else 0.0)
        ep = _rel(pot.cpu().numpy()[rows], phi)
        eg = _rel(grad.cpu().numpy()[rows], g)
        _say(f"[{tag} {kernel}] pot {ep:.2e} grad {eg:.2e}")
        assert ep < tol and eg < tol


@pytest.mark.parametrize("precision,tol", [("bf16x3", 1e-4), ("fp32", 1e-4), ("fp64", 1e-6)])
def test_surface393k_pair_with_the_shipped_entry(surface393k, precision, tol):
    """The benchmark's step as it runs: the package's shipped tuning entry
    for this workload, device and precision (ncrit and tunables), against the
    direct sums on 2,048 sampled rows."""
    torch = require_gpu()
    from paper_2103_01048_amd import FMMPlan, autotune as at
    x, q = surface393k
    xt = torch.tensor(x, device="cuda")
    e = _shipped(at, len(x), 8, precision, xt.device)
    with at.tuning(**{**at.DEFAULTS, **e["tuning"]}):
        plans = [FMMPlan(xt, kernel=k, kappa=KAPPA, p=8, ncrit=e["ncrit"], precision=precision)
                 for k in ("laplace", "yukawa")]
    rows = np.random.default_rng(77).choice(len(x), 2048, replace=False)
    _pair_rows(plans, torch, x, q, rows, tol, f"393k pair {precision} shipped entry ncrit {e['ncrit']}")


@pytest.mark.parametrize("precision,tol", [("fp32", 1e-4), ("fp64", 1e-6)])
@pytest.mark.parametrize("kernel", ["laplace", "yukawa"])
def test_surface393k_fp32_fp64(surface393k, kernel, precision, tol):
    torch = require_gpu()
    from paper_2103_01048_amd import FMMPlan
    x, q = surface393k
    plan = FMMPlan(torch.tensor(x, device="cuda"), kernel=kernel, kappa=KAPPA, p=8, ncrit=128,
                   precision=precision)
    rows = np.random.default_rng(72).choice(len(x), 2048, replace=False)
    _check_rows(plan, torch, x, q, rows, kernel, tol, f"393k {kernel} {precision}")


@pytest.mark.parametrize("kernel", ["laplace", "yukawa"])
def test_batch64_molecules(kernel):
    """The 64-molecule batch in one Laplace and one Yukawa plan evaluated as a
    pair (as the benchmark times it): four molecules (smallest, largest, two
    seeded) against their own direct sums on sampled rows."""
    torch = require_gpu()
    from paper_2103_01048_amd import FMMPlan, eval_pair
    xs, qs = synth.molecule_batch(64, seed=5)
    off = np.concatenate([[0], np.cumsum([len(x) for x in xs])])
    X, Q = np.concatenate(xs), np.concatenate(qs)
    xt = torch.tensor(X, device="cuda")
    plans = [FMMPlan(xt, kernel=k, kappa=KAPPA, p=8, ncrit=128, precision="bf16x3", offsets=off)
             for k in ("laplace", "yukawa")]
    outs = eval_pair(plans[0], plans[1], torch.tensor(Q, device="cuda"))
    pot, grad = outs[0 if kernel == "laplace" else 1]
    pot, grad = pot.cpu().numpy(), grad.cpu().numpy()
    sizes = np.diff(off)
    rng = np.random.default_rng(73)
    pick = sorted({int(np.argmin(sizes)), int(np.argmax(sizes)), *rng.choice(64, 2, replace=False).tolist()})
    kap = KAPPA if kernel == "yukawa" else 0.0
    for m in pick:
        rows = rng.choice(sizes[m], min(512, sizes[m]), replace=False)
        phi, g = D.direct(xs[m][rows], xs[m], qs[m], kernel, kap)
        ep = _rel(pot[off[m] + rows], phi)
        eg = _rel(grad[off[m] + rows], g)
        _say(f"[batch64 {kernel}] molecule {m} ({sizes[m]} points) pot {ep:.2e} grad {eg:.2e}")
        assert ep < 1e-4 and eg < 1e-4


@pytest.mark.parametrize("kernel", ["laplace", "yukawa"])
def test_adjoint_1m_points(kernel):
    """E = 1/2 q.phi on 1,000,002 points, FP32 forward and adjoint: dE/dq =
    phi on sampled rows, dE/dx on 64 seeded coordinates against central
    differences (h = 1e-4 A) of the exact FP64 pair energy."""
    torch = require_gpu()
    from paper_2103_01048_amd import FMMPlan, solvation_style_energy
    x, _ = synth.surface_cloud(500, 333334, seed=81)
    q = np.random.default_rng(81).uniform(-1.0, 1.0, len(x))
    kap = KAPPA if kernel == "yukawa" else 0.0
    plan = FMMPlan(torch.tensor(x, device="cuda"), kernel=kernel, kappa=KAPPA, p=8, ncrit=128, precision="fp32")
    qt = torch.tensor(q, device="cuda", requires_grad=True)
    xt = torch.tensor(x, device="cuda", requires_grad=True)
    solvation_style_energy(plan, qt, xt).backward()
    dq, dx = qt.grad.cpu().numpy(), xt.grad.cpu().numpy()
    rng = np.random.default_rng(82)
    rows = rng.choice(len(x), 2048, replace=False)
    phi, _ = D.direct(x[rows], x, q, kernel, kap)
    edq = _rel(dq[rows], phi)
    pick = rng.choice(len(x), 64, replace=False)
    dims = rng.integers(0, 3, 64)
    h = 1e-4
    fd = np.empty(64)
    for i, (k, d) in enumerate(zip(pick, dims)):
        e = np.zeros(3)
        e[d] = h
        others = np.delete(np.arange(len(x)), k)
        pp, _ = D.direct(x[k:k + 1] + e, x[others], q[others], kernel, kap)
        pm, _ = D.direct(x[k:k + 1] - e, x[others], q[others], kernel, kap)
        fd[i] = q[k] * (pp[0] - pm[0]) / (2 * h)
    edx = _rel(dx[pick, dims], fd)
    _say(f"[adjoint 1M {kernel}] dq {edq:.2e} dx {edx:.2e}")
    assert edq < 1e-4 and edx < 1e-3


@pytest.fixture(scope="module")
def bem2m():
    _say("[fullsize] building the 2M-triangle sphere-union mesh")
    su = synth.sphere_union_spheres(1000, seed=91, box=40.0 * 5.0 ** (1.0 / 3.0))
    v, t = synth.sphere_union_mesh(su, 2_000_000, seed=91, gap=0.5)
    qxyz, q = synth.charges_in_spheres(su, 20000, seed=91)
    return v, t, B.make_mesh(v, t, 3), qxyz, q


def _bem(v, t, precision):
    require_gpu()
    from paper_2103_01048_amd import BEMOperator
    return BEMOperator(v, t, quad_pts=3, eps_in=4.0, eps_out=80.0, kappa=KAPPA, p=8, ncrit=128,
                       precision=precision)


@pytest.mark.parametrize("precision,tol", [("fp32", 1e-4), ("bf16x3", 1e-4), ("fp64", 1e-6)])
def test_bem2m_matvec_and_rhs_rows(bem2m, precision, tol):
    torch = require_gpu()
    v, t, m, qxyz, q = bem2m
    T = len(t)
    op = _bem(v, t, precision)
    rng = np.random.default_rng(92)
    x = rng.standard_normal(2 * T)
    y = op.matvec(torch.tensor(x, device="cuda")).cpu().numpy()
    rows = rng.choice(T, 16, replace=False)
    ref = B.matvec_rows(m, rows, x, 4.0, 80.0, KAPPA)
    e = _rel(np.stack([y[rows], y[T + rows]], axis=1), ref)
    _say(f"[bem 2M {precision}] matvec rows {e:.2e}")
    assert e < tol
    b = op.rhs(qxyz, q).cpu().numpy()
    sub = B.make_mesh(v, t[rows], 3)
    rb = B.rhs(sub, qxyz, q, 4.0)
    er = _rel(np.concatenate([b[rows], b[T + rows]]), rb)
    _say(f"[bem 2M {precision}] rhs rows {er:.2e}")
    assert er < 1e-12


def test_bem2m_gmres_energy(bem2m):
    """GMRES to 1e-6 from the single-precision operator (bf16x3 M2L, as the
    benchmark runs it) with FP64 refinement: the FP64 operator's residual,
    the oracle's residual on sampled rows, and the energy of a sampled
    subset of the charges against the oracle's."""
    torch = require_gpu()
    from paper_2103_01048_amd import gmres
    from paper_2103_01048_amd import _lib
    v, t, m, qxyz, q = bem2m
    T = len(t)
    op32 = _bem(v, t, "bf16x3")
    op64 = _bem(v, t, "fp64")
    b = op32.rhs(qxyz, q)
    x, its, hist, rc = gmres(op32, b, tol=1e-6, maxiter=400, restart=100, refine=op64, inner_tol=1e-4)
    _say(f"[bem 2M gmres] status {rc} iterations {its} estimates "
         + " ".join(f"{h:.1e}" for h in hist[::10]))
    assert rc == _lib.FMM_OK
    r = (b - op64.matvec(x)).norm().item() / b.norm().item()
    _say(f"[bem 2M gmres] FP64 operator residual {r:.2e}")
    assert r <= 1e-6
    xh, bh = x.cpu().numpy(), b.cpu().numpy()
    rng = np.random.default_rng(93)
    rows = rng.choice(T, 16, replace=False)
    ax = B.matvec_rows(m, rows, xh, 4.0, 80.0, KAPPA)
    bref = np.stack([bh[rows], bh[T + rows]], axis=1)
    er = float(np.linalg.norm(ax - bref) / np.linalg.norm(bref))
    _say(f"[bem 2M gmres] oracle residual on 16 rows {er:.2e}")
    assert er < 1e-5
    sel = rng.choice(len(q), 256, replace=False)
    eg = op32.energy(x, qxyz[sel], q[sel])
    eo = B.energy_direct(m, xh, qxyz[sel], q[sel])
    _say(f"[bem 2M energy] 256 charges GPU {eg:.10f} oracle {eo:.10f} kcal/mol")
    assert abs(eg - eo) <= 1e-9 * abs(eo)
    e_all = op32.energy(x, qxyz, q)
    _say(f"[bem 2M energy] all 20,000 charges {e_all:.6f} kcal/mol")
    assert math.isfinite(e_all) and e_all < 0


@pytest.mark.parametrize("kernel", ["laplace", "yukawa"])
def test_shell_30m_points_p10(kernel):
    """30M points on a 30,000-sphere shell (R = 200 A), p = 10, FP32 with the
    bf16x3 M2L, against the direct sum on 512 sampled rows."""
    torch = require_gpu()
    from paper_2103_01048_amd import FMMPlan
    x, q = _shell30m()
    plan = FMMPlan(torch.tensor(x, device="cuda"), kernel=kernel, kappa=KAPPA, p=10, ncrit=128,
                   precision="bf16x3")
    _say(f"[shell 30M {kernel}] setup {plan.info()['setup_ms']:.0f} ms")
    rows = np.random.default_rng(101).choice(len(x), 512, replace=False)
    _check_rows(plan, torch, x, q, rows, kernel, 1e-4, f"shell 30M {kernel} p10")


def test_shell_30m_pair_with_the_shipped_entry():
    """The 30M-point shell's pair evaluation (p = 10) with the shipped tuning
    entry for it, against the direct sums on 256 sampled rows."""
    torch = require_gpu()
    from paper_2103_01048_amd import FMMPlan, autotune as at
    x, q = _shell30m()
    xt = torch.tensor(x, device="cuda")
    e = _shipped(at, len(x), 10, "bf16x3", xt.device)
    with at.tuning(**{**at.DEFAULTS, **e["tuning"]}):
        plans = [FMMPlan(xt, kernel=k, kappa=KAPPA, p=10, ncrit=e["ncrit"], precision="bf16x3")
                 for k in ("laplace", "yukawa")]
    rows = np.random.default_rng(103).choice(len(x), 256, replace=False)
    _pair_rows(plans, torch, x, q, rows, 1e-4, f"shell 30M pair shipped entry ncrit {e['ncrit']}")
    del plans


_SHELL = {}


def _shell30m():
    if "x" not in _SHELL:
        _say("[fullsize] building the 30M-point shell")
        _SHELL["x"] = synth.surface_cloud(30000, 10_000_000, seed=13, shell_radius=200.0)
    return _SHELL["x"]


def test_bem2m_derivative_formulation_solve(bem2m):
    """The derivative formulation on the 2M-triangle mesh: GMRES to 1e-6
    (bf16x3 operator, FP64 refinement), the FP64 operator's residual, and the
    energy of 256 sampled charges against the oracle's for the same
    solution; the energy of all charges agrees with the direct
    formulation's to the discretisation level."""
    torch = require_gpu()
    from paper_2103_01048_amd import BEMOperator, gmres
    from paper_2103_01048_amd import _lib
    v, t, m, qxyz, q = bem2m
    kw = dict(quad_pts=3, eps_in=4.0, eps_out=80.0, kappa=KAPPA, p=8, ncrit=128, formulation="derivative")
    op32 = BEMOperator(v, t, precision="bf16x3", **kw)
    op64 = BEMOperator(v, t, precision="fp64", **kw)
    b = op32.rhs(qxyz, q)
    x, its, hist, rc = gmres(op32, b, tol=1e-6, maxiter=200, restart=100, refine=op64, inner_tol=1e-3)
    _say(f"[bem 2M derivative] status {rc} iterations {its}")
    assert rc == _lib.FMM_OK
    r = (b - op64.matvec(x)).norm().item() / b.norm().item()
    assert r <= 1e-6
    xh = x.cpu().numpy()
    sel = np.random.default_rng(94).choice(len(q), 256, replace=False)
    eg = op32.energy(x, qxyz[sel], q[sel])
    eo = B.energy_direct(m, xh, qxyz[sel], q[sel])
    assert abs(eg - eo) <= 1e-9 * abs(eo)
    e_all = op32.energy(x, qxyz, q)
    _say(f"[bem 2M derivative] residual {r:.2e} energy {e_all:.4f} kcal/mol")
    assert e_all < 0


@pytest.mark.parametrize("formulation", ["derivative", "exterior"])
def test_bem2m_derivative_matvec_rows(bem2m, formulation):
    """bem_matvec of the interior (eq:juffer) and exterior (eq:lu)
    derivative formulations on the 2M-triangle mesh, bf16x3 as the
    benchmark runs it, against oracle rows on 8 sampled triangles."""
    torch = require_gpu()
    from paper_2103_01048_amd import BEMOperator
    v, t, m, qxyz, q = bem2m
    T = len(t)
    op = BEMOperator(v, t, quad_pts=3, eps_in=4.0, eps_out=80.0, kappa=KAPPA, p=8, ncrit=128,
                     precision="bf16x3", formulation=formulation)
    rng = np.random.default_rng(94)
    x = rng.standard_normal(2 * T)
    y = op.matvec(torch.tensor(x, device="cuda")).cpu().numpy()
    rows = rng.choice(T, 8, replace=False)
    ref = B.matvec_rows_derivative(m, rows, x, 4.0, 80.0, KAPPA,
                                   formulation="interior" if formulation == "derivative" else "exterior")
    e = _rel(np.stack([y[rows], y[T + rows]], axis=1), ref)
    _say(f"[bem 2M {formulation} bf16x3] matvec rows {e:.2e}")
    assert e < 1e-4


def test_bem2m_exterior_p1(bem2m):
    """The exterior formulation on P1 elements on the 2M-triangle mesh
    (bf16x3 as the benchmark runs it): bem_matvec against oracle rows on 3
    sampled vertices, then GMRES to 1e-6 with FP64 refinement, the FP64
    operator's residual, and the energy of 256 sampled charges against the
    oracle's for the same solution."""
    torch = require_gpu()
    from oracle import bem_p1 as P1
    from paper_2103_01048_amd import BEMOperator, gmres
    from paper_2103_01048_amd import _lib
    v, t, _, qxyz, q = bem2m
    v, t = synth.used_vertices_only(v, t)
    m = B.make_mesh(v, t, 3)
    nv = len(v)
    kw = dict(quad_pts=3, eps_in=4.0, eps_out=80.0, kappa=KAPPA, p=8, ncrit=128, formulation="exterior_p1")
    op32 = BEMOperator(v, t, precision="bf16x3", **kw)
    rng = np.random.default_rng(95)
    x = rng.standard_normal(2 * nv)
    y = op32.matvec(torch.tensor(x, device="cuda")).cpu().numpy()
    rows = rng.choice(nv, 3, replace=False)
    ref = P1.matvec_rows(m, rows, x, 4.0, 80.0, KAPPA)
    e = _rel(np.stack([y[rows], y[nv + rows]], axis=1), ref)
    _say(f"[bem 2M exterior P1 bf16x3] matvec rows {e:.2e}")
    assert e < 1e-4
    op64 = BEMOperator(v, t, precision="fp64", **kw)
    b = op32.rhs(qxyz, q)
    xs, its, hist, rc = gmres(op32, b, tol=1e-6, maxiter=200, restart=100, refine=op64, inner_tol=1e-3)
    r = (b - op64.matvec(xs)).norm().item() / b.norm().item()
    _say(f"[bem 2M exterior P1] status {rc} iterations {its} residual {r:.2e}")
    assert rc == _lib.FMM_OK and r <= 1e-6
    sel = np.random.default_rng(96).choice(len(q), 256, replace=False)
    eg = op32.energy(xs, qxyz[sel], q[sel])
    eo = P1.energy_direct(m, xs.cpu().numpy(), qxyz[sel], q[sel])
    assert abs(eg - eo) <= 1e-9 * abs(eo)
    e_all = op32.energy(xs, qxyz, q)
    _say(f"[bem 2M exterior P1] energy {e_all:.4f} kcal/mol")
    assert e_all < 0
