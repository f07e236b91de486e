"""bem_rhs_noalloc (the right-hand side with its temporaries in the
library's static device scratch, for callers that cannot allocate) against
bem_rhs, called through the C ABI: two calls in a row, the second on a
smaller mesh with fewer charges, for the direct (P0) and the exterior P1
formulation; bitwise equal results (the same launches in the same order).
Sizes beyond the scratch are refused before any launch."""
import ctypes

import numpy as np
import pytest

import synth
from tests.gpu_util import require_gpu

pytestmark = pytest.mark.gpu


def _call(fn, op, qx, q, out):
    from paper_2103_01048_amd import _lib
    from paper_2103_01048_amd.fmm import _ptr, _stream
    return getattr(_lib.lib(), fn)(op._h, _ptr(qx), _ptr(q), int(q.numel()), _ptr(out), _stream())


@pytest.mark.parametrize("formulation", ["direct", "exterior_p1"])
def test_noalloc_rhs_equals_rhs(formulation):
    torch = require_gpu()
    from paper_2103_01048_amd import BEMOperator, _lib
    for level, nq, seed in ((4, 37, 201), (2, 5, 202)):
        v, t = synth.octa_sphere(level, 4.0)
        print(f"[noalloc] {formulation} triangles={len(t)} charges={nq}", flush=True)
        op = BEMOperator(v, t, quad_pts=3, p=5, ncrit=64, precision="fp64", formulation=formulation)
        rng = np.random.default_rng(seed)
        qx = torch.tensor(rng.uniform(-2.0, 2.0, (nq, 3)), device="cuda")
        q = torch.tensor(rng.uniform(-1.0, 1.0, nq), device="cuda")
        ref = torch.full((2 * op.nu,), float("nan"), dtype=torch.float64, device="cuda")
        got = torch.full_like(ref, float("nan"))
        assert _call("bem_rhs", op, qx, q, ref) == _lib.FMM_OK
        assert _call("bem_rhs_noalloc", op, qx, q, got) == _lib.FMM_OK
        torch.cuda.synchronize()
        assert torch.isfinite(ref).all()
        assert torch.equal(got, ref)


def test_noalloc_rhs_refuses_more_than_its_scratch():
    torch = require_gpu()
    from paper_2103_01048_amd import BEMOperator, _lib
    v, t = synth.octa_sphere(2, 4.0)
    op = BEMOperator(v, t, quad_pts=3, p=4, ncrit=64, precision="fp64")
    qx = torch.zeros((1, 3), dtype=torch.float64, device="cuda")
    q = torch.zeros(1, dtype=torch.float64, device="cuda")
    b = torch.zeros(2 * op.nu, dtype=torch.float64, device="cuda")
    from paper_2103_01048_amd.fmm import _ptr, _stream
    # the size check comes before any launch, so the oversized count is never read
    rc = _lib.lib().bem_rhs_noalloc(op._h, _ptr(qx), _ptr(q), _lib.BEM_RHS_SCRATCH_DOUBLES, _ptr(b), _stream())
    assert rc == _lib.FMM_EINVAL
    assert "scratch" in _lib.lib().fmm_last_error().decode()
