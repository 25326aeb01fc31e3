"""Differentiable sampling: x as a function of the real weights.

Forward: quantise the weights (per distribution), build the forest, sample.
Backward: the library's adjoint kernel gives dL/dv for the continuous position
x of Sec. 5 with the sampled index held fixed; autograd then chains whatever
produced v (e.g. a softplus of logits).
"""
from __future__ import annotations

import torch

from . import (RTF_ERR_VALUE, RtfError, backward, build_batched, cells_like, quantize,
               sample_batched)


class RTFSample(torch.autograd.Function):
    """x = RTFSample.apply(v, u, elem_off, sample_off, cell_ratio)
       x = RTFSample.apply(v, u, plan)

    v           float32[n_total] non-negative weights (requires_grad allowed)
    u           uint64[S] uniforms; sample_off int64[D+1] splits them by
                distribution; elem_off int64[D+1] splits v
    cell_ratio  guide cells per weight (m_d = round(ratio * n_d), at least 1)
    plan        a plan.DiffPlan for these shapes: every buffer preallocated,
                nothing read back, so forward and backward can be captured
                in a HIP graph; x is then a view of the plan's buffer
    Returns x float64[S].

    Without a plan the forward raises RtfError on a negative, NaN or
    infinite weight (RTF_ERR_VALUE) and on a distribution whose weights are
    all zero (RTF_ERR_ZERO_TOTAL); it synchronises for that, as it does to
    size the workspace.  With a plan nothing is read back: call
    plan.check() to raise on the same errors.
    """

    @staticmethod
    def forward(ctx, v, u, elem_off, sample_off=None, cell_ratio=1.0):
        from .plan import DiffPlan
        if isinstance(elem_off, DiffPlan):
            plan = elem_off
            _, x = plan.run(v.detach(), u)
            ctx.plan = plan
            ctx.save_for_backward(u)
            return x.view(-1)
        status = torch.zeros(1, dtype=torch.int32, device=v.device)
        q, scale = quantize(v.detach().contiguous(), elem_off, status=status)
        f = build_batched(q, elem_off, cells_like(elem_off, cell_ratio))
        if int(status.item()) & (1 << RTF_ERR_VALUE):
            raise RtfError(RTF_ERR_VALUE, "rtf_quantize_f32")
        f.check()
        idx, x = sample_batched(f, sample_off, u, want_x=True)
        ctx.plan = None
        ctx.forest = f
        ctx.save_for_backward(u, idx, scale, sample_off)
        ctx.v_dtype = v.dtype
        return x

    @staticmethod
    def backward(ctx, grad_x):
        if ctx.plan is not None:
            (u,) = ctx.saved_tensors
            g = ctx.plan.backward(u, grad_x.contiguous())
            return g, None, None, None, None
        u, idx, scale, sample_off = ctx.saved_tensors
        g = backward(ctx.forest, u, idx, grad_x.contiguous().to(torch.float64), scale,
                     sample_off=sample_off)
        return g.to(ctx.v_dtype), None, None, None, None
