"""HIP graph capture of the hot path: one fmm_eval_pair step (which forks
its far-field passes to a side stream and joins them back) and one
bem_matvec (P0 direct and P1 exterior) are captured with torch.cuda.graph and replayed several times,
with eager work and synchronisation between the replays; every replay must
equal the eager result bitwise (the evaluation is deterministic and records
no memset or allocation)."""
import numpy as np
import pytest

import synth
from tests.gpu_util import require_gpu

pytestmark = pytest.mark.gpu


def _capture(torch, fn):
    s = torch.cuda.Stream()
    s.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(s):
        for _ in range(2):
            fn()
    torch.cuda.current_stream().wait_stream(s)
    torch.cuda.synchronize()
    g = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g):
        out = fn()
    torch.cuda.synchronize()
    return g, out


def test_pair_step_graph_replays_equal_eager():
    torch = require_gpu()
    from paper_2103_01048_amd import FMMPlan, eval_pair
    su = synth.sphere_union_spheres(30, seed=131, box=14.0)
    v, t = synth.sphere_union_mesh(su, 6000, seed=131)
    x = synth.three_point_cloud(v, t)
    xt = torch.tensor(x, device="cuda")
    a = FMMPlan(xt, kernel="laplace", p=6, ncrit=64, precision="bf16x3")
    b = FMMPlan(xt, kernel="yukawa", kappa=0.125, p=6, ncrit=64, precision="bf16x3")
    q = torch.tensor(np.random.default_rng(131).standard_normal(len(x)), device="cuda", dtype=torch.float32)
    (ra, ga), (rb, gb) = eval_pair(a, b, q)
    ref = [u.clone() for u in (ra, ga, rb, gb)]
    g, out = _capture(torch, lambda: eval_pair(a, b, q))
    for _ in range(3):
        g.replay()
        torch.cuda.synchronize()
        got = [out[0][0], out[0][1], out[1][0], out[1][1]]
        assert all(torch.equal(u, w) for u, w in zip(got, ref))
        eval_pair(a, b, q)
        torch.cuda.synchronize()


@pytest.mark.parametrize("formulation", ["direct", "exterior_p1"])
def test_bem_matvec_graph_replays_equal_eager(formulation):
    torch = require_gpu()
    from paper_2103_01048_amd import BEMOperator
    v, t = synth.octa_sphere(4, 4.0)
    op = BEMOperator(v, t, quad_pts=3, p=6, ncrit=64, precision="fp32", formulation=formulation)
    x = torch.tensor(np.random.default_rng(132).standard_normal(2 * op.nu), device="cuda")
    ref = op.matvec(x).clone()
    g, out = _capture(torch, lambda: op.matvec(x))
    for _ in range(3):
        g.replay()
        torch.cuda.synchronize()
        assert torch.equal(out, ref)
        op.matvec(x)
        torch.cuda.synchronize()
