"""Learnable bandwidth on top of ``flsq_bandwidth_loss_grad`` (the reparameterisation appendix).

The features are frozen base draws What_j with biases b_j; the weights used are W_j = L What_j
with L lower triangular (the anisotropic covariance L L^T), or L = sigma I for the scalar
bandwidth.  Each evaluation re-solves the regularised least-squares problem exactly on the GPU
and returns the outer loss ||A(L) beta* - b||^2 with its gradient in L; the outer optimiser is
AdamW with decoupled weight decay (the paper's hybrid training procedure) over the d(d+1)/2 (or
one) parameters, each step one ``flsq_adam_step`` on the device; the parameters come back to the
host only to form L for the next evaluation.
"""
from __future__ import annotations

import numpy as np

from . import fastlsq as fl


def lower_pairs(d):
    """(p, q), q <= p, in the packed row-by-row order of the gradient."""
    return [(p, q) for p in range(d) for q in range(p + 1)]


class LearnableBandwidth:
    """ctx: a fastlsq Context; base: a Basis over the frozen draws What (device n x d) and b;
    rows: the stacked operator rows with data; opts: the inner solve's options."""

    def __init__(self, ctx, base: fl.Basis, rows: fl.Rows, opts, d, scalar=True):
        import torch
        self.ctx, self.base, self.rows, self.opts, self.d = ctx, base, rows, opts, int(d)
        self.scalar = bool(scalar)
        self.pairs = lower_pairs(self.d)
        self.beta = torch.empty(base.W.shape[0], dtype=torch.float64, device=base.W.device)

    def L_of(self, params):
        params = np.atleast_1d(np.asarray(params, dtype=np.float64))
        if self.scalar:
            return params[0] * np.eye(self.d)
        L = np.zeros((self.d, self.d))
        for k, (p, q) in enumerate(self.pairs):
            L[p, q] = params[k]
        return L

    def params_of(self, L):
        L = np.asarray(L, dtype=np.float64)
        if self.scalar:
            return np.array([L[0, 0]])
        return np.array([L[p, q] for p, q in self.pairs])

    def loss_and_grad(self, params):
        """Outer loss and its gradient in the parameters (sigma, or the packed entries of L);
        beta* of this evaluation stays in ``self.beta``."""
        loss, g = fl.flsq_bandwidth_loss_grad(self.ctx, self.base, self.L_of(params), self.rows, self.opts, self.beta)
        if self.scalar:
            g = np.array([sum(g[k] for k, (p, q) in enumerate(self.pairs) if p == q)])
        return loss, g

    def fit_adamw(self, params0, steps=80, lr=0.1, betas=(0.9, 0.999), eps=1e-8, weight_decay=0.01):
        """AdamW (p <- p (1 - lr wd), then the bias-corrected Adam step) by ``flsq_adam_step``.
        Returns the parameters and the loss at the start of every step, and the final parameters."""
        import torch
        dev = self.beta.device
        p = torch.tensor(np.atleast_1d(np.asarray(params0, dtype=np.float64)), dtype=torch.float64, device=dev)
        m = torch.zeros_like(p)
        v = torch.zeros_like(p)
        b1, b2 = betas
        hist_p, hist_loss = [], []
        for t in range(1, steps + 1):
            ph = p.cpu().numpy()
            loss, g = self.loss_and_grad(ph)
            hist_p.append(ph.copy())
            hist_loss.append(loss)
            gt = torch.tensor(g, dtype=torch.float64, device=dev)
            fl.flsq_adam_step(self.ctx, p, gt, m, v, t, lr, b1, b2, eps, weight_decay=weight_decay)
        return np.array(hist_p), np.array(hist_loss), p.cpu().numpy()
