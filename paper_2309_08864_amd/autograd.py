"""torch.autograd binding of the out-of-core adjoint.

StencilLoss.apply(u0, w, target, spec) returns L = 1/2 ||u_T - target||^2
(FP64 scalar) where u_T is the out-of-core sweep of u0 with weights w;
backward gives dL/du0 and dL/dw from the library's adjoint sweep (computed
together with the loss in forward and scaled by the incoming gradient).
u0 and target are pinned host tensors; spec holds the Plan arguments other
than the weights (grid, stencil, T, tb_depth, chunks, budget, ...) plus
'ckpt_every'."""
import numpy as np
import torch

from .plan import Plan


class StencilLoss(torch.autograd.Function):
    @staticmethod
    def forward(ctx, u0, w, target, spec):
        spec = dict(spec)
        ckpt_every = spec.pop("ckpt_every")
        plan = Plan(weights=[float(x) for x in w.detach().double().cpu().numpy()], adjoint=True,
                    **spec).bind()
        try:
            loss, gu, gw, _ = plan.adjoint(u0.detach(), target.detach(), ckpt_every)
        finally:
            plan.close()
        ctx.save_for_backward(gu, torch.from_numpy(np.ascontiguousarray(gw)))
        ctx.w_dtype = w.dtype
        return torch.tensor(loss, dtype=torch.float64)

    @staticmethod
    def backward(ctx, g):
        gu, gw = ctx.saved_tensors
        g = g.detach().cpu().double()
        grad_u0 = (gu.double() * g).to(gu.dtype) if ctx.needs_input_grad[0] else None
        grad_w = (gw * g).to(ctx.w_dtype) if ctx.needs_input_grad[1] else None
        return grad_u0, grad_w, None, None
