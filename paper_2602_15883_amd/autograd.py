"""torch.autograd.Function over the fused step.

The forward runs pinn_step without the Adam update (PINN_NO_UPDATE): the HIP
kernels evaluate every subdomain's loss (section 2.2, final local objective)
and, through the hand-written adjoint of the derivative-carrying forward, its
exact gradient.  The backward returns that gradient scaled by the incoming
gradient; nothing is differentiated by PyTorch.  The parameter tensors passed
in must be the context's own theta tensors, so that an optimizer updating them
in place changes what the next forward sees.
"""
from __future__ import annotations

import torch

from .context import Context


class PinnLoss(torch.autograd.Function):
    @staticmethod
    def forward(fctx, ctx: Context, *thetas):
        for s, th in enumerate(thetas):
            if th.data_ptr() != ctx.subs[s].theta.data_ptr():
                raise ValueError("PinnLoss needs the context's own theta tensors")
        loss, g = ctx.step(1, update=False, want_grad=True)
        fctx.save_for_backward(g)
        fctx.n_sub = len(thetas)
        return loss[:, 6].clone()

    @staticmethod
    def backward(fctx, grad_loss):
        (g,) = fctx.saved_tensors
        grads = [grad_loss[s] * g[s] for s in range(fctx.n_sub)]
        return (None, *grads)


def pinn_loss(ctx: Context) -> torch.Tensor:
    """Per-subdomain total losses [n_sub] with gradients to the context's theta
    tensors (which must have requires_grad set)."""
    return PinnLoss.apply(ctx, *[s.theta for s in ctx.subs])
