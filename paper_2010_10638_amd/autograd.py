"""Tucker completion loss as a torch.autograd.Function over the HIP adjoint TTMc.

The forward call runs ``ttmc_adjoint`` once: it returns the loss and, from the same pass over the
entries, the gradients with respect to the core and every factor; backward only scales them by
the incoming gradient.  Marshalling only - the arithmetic is in the library.
"""
from __future__ import annotations

import torch

from . import binding


class TuckerCompletionLoss(torch.autograd.Function):
    """loss(G, U_1..U_N) = sum_p (xhat_p - x_p)^2 / (2 |Omega|) over the entries of ``tctx``."""

    @staticmethod
    def forward(fctx, tctx, G, *U):
        loss, gG, gU = binding.ttmc_adjoint(tctx, G.contiguous(), [u.contiguous() for u in U])
        fctx.save_for_backward(gG, *gU)
        return loss.reshape(())

    @staticmethod
    def backward(fctx, grad):
        gG, *gU = fctx.saved_tensors
        return (None, grad * gG, *[grad * g for g in gU])


def completion_loss(tctx, G: torch.Tensor, U) -> torch.Tensor:
    """Differentiable completion loss; G: [R_1..R_N], U[k]: [I_k, R_k] in the context's type."""
    return TuckerCompletionLoss.apply(tctx, G, *U)
