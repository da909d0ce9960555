"""torch.autograd.Function wrappers over the C ABI.  torch supplies device memory and the
stream; the products, solves and their adjoints run in libddf's kernels.

SpMVFn.apply(values, x, plan)  -> y = A x          (grad: values, x)
SpTRSVFn.apply(values, b, plan) -> x with L x = b  (grad: values, b)
x / b may be 1-D (one right-hand side) or (n, k) with k <= 32, float64, on the GPU.
"""
from __future__ import annotations

import torch

from . import ddf


def _as2d(t):
    return (t.unsqueeze(1) if t.dim() == 1 else t).contiguous()


class SpMVFn(torch.autograd.Function):
    @staticmethod
    def forward(ctx, values, x, plan):
        x2 = _as2d(x)
        k = x2.shape[1]
        y = torch.empty((plan.n_rows, k), dtype=torch.float64, device=x.device)
        ddf.ddf_spmv_v(plan, values.contiguous(), x2, y, k)
        ctx.plan, ctx.one = plan, x.dim() == 1
        ctx.save_for_backward(values, x2)
        return y.squeeze(1) if ctx.one else y

    @staticmethod
    def backward(ctx, gy):
        values, x2 = ctx.saved_tensors
        g = _as2d(gy)
        k = x2.shape[1]
        gx = torch.empty_like(x2) if ctx.needs_input_grad[1] else None
        gv = torch.empty_like(values) if ctx.needs_input_grad[0] else None
        if gx is not None or gv is not None:
            ddf.ddf_spmv_adjoint(ctx.plan, values.contiguous(), x2, g, gx, gv, k)
        if gx is not None and ctx.one:
            gx = gx.squeeze(1)
        return gv, gx, None


class SpTRSVFn(torch.autograd.Function):
    @staticmethod
    def forward(ctx, values, b, plan):
        b2 = _as2d(b)
        k = b2.shape[1]
        x = torch.empty_like(b2)
        ddf.ddf_sptrsv_v(plan, values.contiguous(), b2, x, k)
        ctx.plan, ctx.one = plan, b.dim() == 1
        ctx.save_for_backward(values, x)
        return x.squeeze(1) if ctx.one else x

    @staticmethod
    def backward(ctx, gx):
        values, x = ctx.saved_tensors
        g = _as2d(gx)
        k = x.shape[1]
        gb = torch.empty_like(x)
        gv = torch.empty_like(values) if ctx.needs_input_grad[0] else None
        ddf.ddf_sptrsv_adjoint(ctx.plan, values.contiguous(), x, g, gb, gv, k)
        gb = gb if ctx.needs_input_grad[1] else None
        if gb is not None and ctx.one:
            gb = gb.squeeze(1)
        return gv, gb, None


def spmv(plan, values, x):
    return SpMVFn.apply(values, x, plan)


def sptrsv(plan, values, b):
    return SpTRSVFn.apply(values, b, plan)
