"""torch.autograd.Function over the library's ELBO (the adjoint kernel of the pixel path).

forward:  cel_elbo_eval -- saves only theta
backward: cel_elbo_grad at the saved theta (pixel terms are recomputed, not stored),
          scaled by the incoming gradient
"""
import torch

from . import api


class ElboFunction(torch.autograd.Function):
    @staticmethod
    def forward(ctx, theta, plan):
        tot, _ = api.elbo_eval(plan, theta.detach())
        ctx.save_for_backward(theta)
        ctx.plan = plan
        return tot.reshape(())

    @staticmethod
    def backward(ctx, grad_out):
        theta, = ctx.saved_tensors
        _, _, g = api.elbo_grad(ctx.plan, theta.detach())
        return grad_out * g.to(theta.dtype), None


def elbo(plan, theta):
    """Global ELBO of `plan` at theta [S,32] (float64 cuda) as a differentiable scalar."""
    return ElboFunction.apply(theta, plan)
