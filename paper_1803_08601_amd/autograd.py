"""torch.autograd.Function over the library: C = A B with gradients for A's
values and for B (L = <dC, C>): dvals = SDDMM(dC, B) on A's pattern and
dB = A^T dC through the plan's once-built transpose. Every step runs in the
HIP library; torch only provides memory and the stream."""
import torch

from . import native as nv


class SpMMFunction(torch.autograd.Function):
    @staticmethod
    def forward(ctx, plan, vals, B):
        C = torch.empty(plan.m, plan.ld, dtype=torch.float32, device=B.device)
        plan.execute(vals, B, C)
        ctx.plan = plan
        ctx.save_for_backward(vals, B)
        return C[:, :plan.n] if plan.ld != plan.n else C

    @staticmethod
    def backward(ctx, dC):
        plan = ctx.plan
        vals, B = ctx.saved_tensors
        dC = dC.to(torch.float32)
        if plan.ld != plan.n or not dC.is_contiguous():
            full = torch.zeros(plan.m, plan.ld, dtype=torch.float32, device=dC.device)
            full[:, :plan.n] = dC
            dC = full
        dvals = dB = None
        if ctx.needs_input_grad[1]:
            dv = torch.empty(plan.nnz, dtype=torch.float32, device=dC.device)
            plan.sddmm(dC, B, dv)
            dvals = dv.to(vals.dtype)
        if ctx.needs_input_grad[2]:
            if not plan.info().has_transpose:
                plan.transpose_build()
            db = torch.empty(plan.k, plan.ld, dtype=torch.float32, device=dC.device)
            plan.execute_t(vals, dC, db)
            db = db[:, :plan.n] if plan.ld != plan.n else db
            dB = db.to(B.dtype)
        return None, dvals, dB


def spmm(plan, vals, B):
    """C = A B (float32) for the structure held by ``plan``; differentiable in
    ``vals`` and ``B``."""
    return SpMMFunction.apply(plan, vals, B)
