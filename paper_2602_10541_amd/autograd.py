"""torch.autograd.Function over the library's adjoint (gradients through the pre-factored solve).

Section 2.5: the forward map (theta, kappa) -> predicted observations passes through one
factored Tikhonov solve, so the gradient of a data misfit needs one more solve with the
same factor plus the analytic derivative of A in the operator coefficient kappa.
``flsq_inverse_loss_grad`` computes the per-hypothesis misfit and both gradients in one
call; this Function exposes them to autograd (the backward only scales the stored
gradients by the incoming cotangent).
"""
from __future__ import annotations

import torch

from . import fastlsq as fl


class InverseProblem:
    """A factored heat-source system plus observation geometry (all device tensors).

    ``kappa`` is the operator coefficient the factor was built for.  ``refactor(kappa)``, when
    given, returns a new factor for another kappa (the system matrix depends on kappa, so a new
    kappa needs a new factorisation); without it the problem accepts only its own kappa.

    ``cache_observations``: keep the observation operator R = H (A^T A + mu I)^{-1} A_src^T on
    the factor (n_obs refined solves, once per factor), so that calls without the kappa
    gradient are two products with R instead of two refined solves.
    """

    def __init__(self, ctx, factor, n_src_rows, src_weight, n_lap_dims, x_obs, data, kappa=None, refactor=None,
                 cache_observations=False):
        self.ctx, self.F = ctx, factor
        self.n_src_rows, self.src_weight, self.n_lap_dims = int(n_src_rows), float(src_weight), int(n_lap_dims)
        self.x_obs = x_obs.contiguous()
        self.data = data.contiguous()
        self.kappa = None if kappa is None else float(kappa)
        self.refactor = refactor
        self.cache_observations = bool(cache_observations)
        if self.cache_observations:
            fl.flsq_inverse_prepare(self.ctx, self.F, self.n_src_rows, self.x_obs)

    def set_kappa(self, kappa):
        kappa = float(kappa)
        if self.kappa is not None and kappa == self.kappa:
            return
        if self.refactor is None:
            raise ValueError(f"the factor was built for kappa = {self.kappa}; kappa = {kappa} needs a refactor callable")
        self.F = self.refactor(kappa)
        self.kappa = kappa
        if self.cache_observations:
            fl.flsq_inverse_prepare(self.ctx, self.F, self.n_src_rows, self.x_obs)

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
    """loss[h] = mean_k (H beta(theta_h, kappa) - d)_k^2 with beta from the factored solve.

    thetas: K x 4 (a, c_x, c_y, w) per hypothesis; kappa: a one-element tensor, the diffusion
    coefficient of the interior operator d/dt - kappa Laplace_x, shared by the K hypotheses.
    The backward returns dL/dtheta (K x 4, row h scaled by the cotangent of loss[h]) and
    dL/dkappa = sum_h cotangent_h dL_h/dkappa (kappa's shape).
    """

    @staticmethod
    def forward(ctx, thetas, kappa, problem: InverseProblem):
        problem.set_kappa(float(kappa.detach().reshape(-1)[0]))
        loss, g, gk = problem.loss_and_grad(thetas.detach(), want_kappa=True)
        ctx.kappa_shape = kappa.shape
        ctx.save_for_backward(g, gk)
        return loss

    @staticmethod
    def backward(ctx, grad_loss):
        g, gk = ctx.saved_tensors
        dk = (grad_loss * gk).sum().reshape(ctx.kappa_shape)
        return grad_loss[:, None] * g, dk, None
