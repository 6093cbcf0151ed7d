"""Poisson log-likelihood as a torch.autograd.Function over the library's
hand-written adjoint (no torch arithmetic on the hot path).

    loss = PoissonLLK.apply(obj, probe, plan)      # 0-dim float64 tensor
    loss.backward()                                # obj.grad, probe.grad

The gradient follows PyTorch's complex convention dL/dRe + i dL/dIm, which is
what the library's ptycho_ml_grad returns.
"""
from __future__ import annotations

import torch


class PoissonLLK(torch.autograd.Function):
    @staticmethod
    def forward(ctx, obj: torch.Tensor, probe: torch.Tensor, plan) -> torch.Tensor:
        need = ctx.needs_input_grad[0] or ctx.needs_input_grad[1]
        if need:
            # one pass gives the LLK and both gradients
            g_obj, g_probe, llk = plan.ml_grad(obj.detach(), probe.detach())
            ctx.save_for_backward(g_obj, g_probe)
        else:
            llk = plan.llk(obj.detach(), probe.detach())
        return llk[0].clone()

    @staticmethod
    def backward(ctx, grad_out: torch.Tensor):
        g_obj, g_probe = ctx.saved_tensors
        s = grad_out.to(torch.float32)
        go = g_obj * s if ctx.needs_input_grad[0] else None
        gp = g_probe * s if ctx.needs_input_grad[1] else None
        return go, gp, None


def poisson_llk(obj: torch.Tensor, probe: torch.Tensor, plan) -> torch.Tensor:
    return PoissonLLK.apply(obj, probe, plan)
