"""torch.autograd.Function over the library's adjoint (gradients through the pre-factored solve).

Section 2.5: the forward map theta -> predicted observations passes through one
factored Tikhonov solve, so the gradient of a data misfit needs one more solve
with the same factor.  ``flsq_inverse_loss_grad`` computes the per-hypothesis
misfit and both gradients in one call; this Function exposes it to autograd
(the backward only scales the stored gradients by the incoming cotangent).
"""
from __future__ import annotations

import torch

from . import fastlsq as fl


class InverseProblem:
    """A factored heat-source system plus observation geometry (all device tensors)."""

    def __init__(self, ctx, factor, n_src_rows, src_weight, n_lap_dims, x_obs, data):
        self.ctx, self.F = ctx, factor
        self.n_src_rows, self.src_weight, self.n_lap_dims = int(n_src_rows), float(src_weight), int(n_lap_dims)
        self.x_obs = x_obs.contiguous()
        self.data = data.contiguous()

    def loss_and_grad(self, thetas, want_kappa=True):
        K = thetas.shape[0]
        dev = thetas.device
        loss = torch.empty(K, dtype=torch.float64, device=dev)
        g = torch.empty((K, 4), dtype=torch.float64, device=dev)
        gk = torch.empty(K, dtype=torch.float64, device=dev) if want_kappa else None
        fl.flsq_inverse_loss_grad(self.ctx, self.F, self.n_src_rows, self.src_weight, self.n_lap_dims,
                                  thetas.contiguous(), self.x_obs, self.data, loss, g, gk)
        return loss, g, gk


class InverseSolve(torch.autograd.Function):
    """loss[h] = mean_k (H beta(theta_h) - d)_k^2 with beta(theta) from the factored solve."""

    @staticmethod
    def forward(ctx, thetas, problem: InverseProblem):
        loss, g, _ = problem.loss_and_grad(thetas.detach(), want_kappa=False)
        ctx.save_for_backward(g)
        return loss

    @staticmethod
    def backward(ctx, grad_loss):
        (g,) = ctx.saved_tensors
        return grad_loss[:, None] * g, None
