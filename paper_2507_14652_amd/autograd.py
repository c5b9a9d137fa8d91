"""The masked potential as a differentiable PyTorch function.

U(Theta_s) of every chain (Sec. 3.2, with the Gaussian likelihood and prior
of App. C) is evaluated by the engine's forward kernels, and its gradient
with respect to the selected entries by the engine's hand-written adjoint
kernels (the same ones the leapfrog uses).  PyTorch only sees a function
from the positions of all chains to their potentials.
"""

from __future__ import annotations

import torch


class MaskedPotential(torch.autograd.Function):
    """forward(theta_s [nnz], sampler) -> U [n_chains] (float64): sets the
    engine's positions to theta_s (so the engine state changes, as
    Sampler.set_state does) and returns the potential of every chain.
    backward: grad_out[c] * dU_c/dtheta_s over chain c's entries.

    FP64 and FP32 engines: backward is the derivative of forward (the same
    products).  BF16 and split-BF16 engines: forward returns U from their
    FP32 energy pass and backward the gradient of their BF16 products, the
    quantities the leapfrog and the Metropolis test of those engines use; so
    backward equals the derivative of forward only up to the gradient error
    of the BF16 products (about 1e-2 relative for BF16, 1e-5 for split
    BF16)."""

    @staticmethod
    def forward(ctx, theta_s, sampler):
        sampler.set_state(theta_s.detach())
        U, g = sampler.grad()
        counts = torch.as_tensor(sampler.offs[1:] - sampler.offs[:-1], device=g.device)
        ctx.save_for_backward(g, counts)
        ctx.in_dtype = theta_s.dtype
        return torch.as_tensor(U, dtype=torch.float64, device=theta_s.device)

    @staticmethod
    def backward(ctx, grad_out):
        g, counts = ctx.saved_tensors
        scale = torch.repeat_interleave(grad_out.to(device=g.device, dtype=g.dtype), counts)
        return (scale * g).to(ctx.in_dtype), None


def masked_potential(theta_s, sampler):
    """U of every chain at theta_s, differentiable in theta_s."""
    return MaskedPotential.apply(theta_s, sampler)
