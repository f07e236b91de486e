"""torch.autograd.Function around fmm_eval with the hand-written adjoint
(fmm_adjoint): densities and point positions both receive gradients.

    pot = fmm_potential(plan, q, xyz)

`xyz` must hold the points the plan was built from (the plan holds the tree
and translation operators for those points; forward raises ValueError
otherwise, FMMPlan.check_points); its gradient is
  dL/dx_k = sum_c gbar_ck grad(phi_c)_k + q_ck grad(psi_c)_k,  psi = G gbar,
and the density gradient is G gbar (the kernel is symmetric)."""
from __future__ import annotations

import ctypes

import torch

from ._lib import check, lib
from .fmm import FMMPlan, _ptr, _stream


class FMMPotential(torch.autograd.Function):
    @staticmethod
    def forward(ctx, q, xyz, plan: FMMPlan):
        if xyz is not None:
            plan.check_points(xyz)
        squeeze = q.ndim == 1
        qq = (q.reshape(1, -1) if squeeze else q).to(plan.dtype).contiguous()
        pot, grad = plan.eval(qq, gradient=True)
        ctx.plan = plan
        ctx.squeeze = squeeze
        ctx.q_dtype = q.dtype
        ctx.x_dtype = xyz.dtype if xyz is not None else plan.dtype
        ctx.save_for_backward(qq, grad)
        return pot[0] if squeeze else pot

    @staticmethod
    def backward(ctx, gpot):
        plan: FMMPlan = ctx.plan
        qq, grad = ctx.saved_tensors
        gb = (gpot.reshape(1, -1) if ctx.squeeze else gpot).to(plan.dtype).contiguous()
        nrhs = qq.shape[0]
        need_q = ctx.needs_input_grad[0]
        need_x = len(ctx.needs_input_grad) > 1 and ctx.needs_input_grad[1]
        dq = torch.empty_like(qq) if need_q else None
        dx = torch.empty((plan.n, 3), dtype=plan.dtype, device=qq.device) if need_x else None
        if need_q or need_x:
            check(lib().fmm_adjoint(plan._h, _ptr(qq), _ptr(gb), _ptr(grad), nrhs, _ptr(dq), _ptr(dx), _stream()),
                  "fmm_adjoint")
        if dq is not None:
            dq = (dq[0] if ctx.squeeze else dq).to(ctx.q_dtype)
        if dx is not None:
            dx = dx.to(ctx.x_dtype)
        return dq, dx, None


def fmm_potential(plan: FMMPlan, q, xyz=None):
    """Differentiable FMM potential (targets = sources = the plan's points).
    xyz: None (no position gradient) or the plan's points, which then
    receive dE/dx."""
    return FMMPotential.apply(q, xyz, plan)


def solvation_style_energy(plan: FMMPlan, q, xyz=None):
    """E = 1/2 q . phi(q): the quadratic form whose gradients are phi and
    q grad(phi)."""
    pot = fmm_potential(plan, q, xyz)
    return 0.5 * (q.to(pot.dtype) * pot).sum()
