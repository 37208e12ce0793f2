"""``torch.autograd.Function`` view of the PWF loss (Eq. 2) on a batch.

The forward pass returns the per-instance loss (the library's forward model
and misfit only); only psi is saved.  The backward pass calls the library
again, recomputing every forward field, and
returns dL/dRe psi + i dL/dIm psi, which is torch's gradient convention for a
real function of complex inputs.  Memory per instance is therefore one complex
field (psi) between the two passes, however large the batch.
"""

from __future__ import annotations

import torch

from .api import PWF


class PWFLoss(torch.autograd.Function):
    @staticmethod
    def forward(ctx, psi: torch.Tensor, batch: PWF, y: tuple):
        if psi.dim() != 3 or psi.dtype != torch.complex64:
            raise ValueError("psi must be a complex64 tensor of shape (n, ny, nx)")
        parts = [psi[i] for i in range(psi.shape[0])]
        loss, _, _ = batch.gradient(parts, list(y), want_g=False, want_d=False)
        ctx.batch = batch
        ctx.y = y
        ctx.save_for_backward(psi)
        return loss

    @staticmethod
    def backward(ctx, grad_loss: torch.Tensor):
        (psi,) = ctx.saved_tensors
        parts = [psi[i] for i in range(psi.shape[0])]
        g = torch.empty_like(psi)   # one buffer; the library writes each instance's slice
        ctx.batch.loss_grad(parts, list(ctx.y), grad_out=[g[i] for i in range(psi.shape[0])])
        g.mul_(grad_loss.to(torch.float32).reshape(-1, 1, 1))
        return g, None, None


def pwf_loss(psi: torch.Tensor, batch: PWF, y) -> torch.Tensor:
    """Differentiable per-instance loss of a (n, ny, nx) complex64 batch of psi."""
    return PWFLoss.apply(psi, batch, tuple(y))
