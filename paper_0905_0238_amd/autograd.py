"""Differentiable solve: V~ = EDTSolve.apply(d_rows, lambda_rel, vel, plan).

Forward: green -> assemble -> solve in FP64 (paper, Section 2.1).  Backward:
the library's hand-written adjoint (edt_adjoint) with respect to the data
rows, the relative damping lambda_rel and the layer velocities; the Green's
tables are recomputed from the velocities rather than kept from the forward
pass, and the evanescent-cut mask of the plan is held fixed.  Gradients of
complex tensors follow PyTorch's convention dL/dRe + i dL/dIm.
"""
from __future__ import annotations

import torch

__all__ = ["EDTSolve", "edt_solve"]


class EDTSolve(torch.autograd.Function):
    @staticmethod
    def forward(ctx, d_rows, lambda_rel, vel, plan):
        lam = float(lambda_rel)
        d = d_rows.detach().to(device=plan.device, dtype=plan.data_dtype).contiguous()
        vl = vel.detach().to(device=plan.device, dtype=torch.float64).contiguous()
        g64, _ = plan.green(vl, want32=False)
        gram, rhs, trace = plan.assemble(g64, None, d, "fp64")
        x, v, info, _ = plan.solve(g64, d, gram, rhs, trace, lam)
        del g64, rhs
        ctx.plan, ctx.lam = plan, lam
        ctx.save_for_backward(d, vl, gram, trace, x, info)
        return v

    @staticmethod
    def backward(ctx, grad_v):
        d, vl, chol, trace, x, info = ctx.saved_tensors
        need_d, need_l, need_v = ctx.needs_input_grad[:3]
        plan = ctx.plan
        g64, _ = plan.green(vl, want32=False)   # recomputed, not stored
        gd, gl, gvel = plan.adjoint(vl, g64, d, chol, trace, x, ctx.lam, grad_v.contiguous(),
                                    want_d=need_d, want_lambda=need_l, want_vel=need_v)
        gl = gl.reshape(()) if gl is not None else None
        return gd, gl, gvel, None


def edt_solve(d_rows, lambda_rel, vel, plan):
    """Functional form of EDTSolve.apply; lambda_rel and vel may require grad."""
    if not torch.is_tensor(lambda_rel):
        lambda_rel = torch.tensor(float(lambda_rel), dtype=torch.float64, device=plan.device)
    return EDTSolve.apply(d_rows, lambda_rel, vel, plan)
