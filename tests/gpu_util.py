"""Shared helpers for the GPU tests (device setup, problem transfer, error metrics)."""
import math

import numpy as np
import pytest


def require_gpu():
    torch = pytest.importorskip("torch")
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2602_10541_amd import fastlsq
    return torch, fastlsq


_CTX = {}


def context():
    torch, fl = require_gpu()
    if "ctx" not in _CTX:
        _CTX["ctx"] = fl.Context(0)
    return _CTX["ctx"]


def amplitude_bound(W, terms, weight, normalize=True):
    """Per-feature bound |weight| * norm * sum_t |c_t| |W^alpha_t| on |A_ij| (scale of the entry error)."""
    n, d = W.shape
    s = np.zeros(n)
    for c, a in terms:
        mono = np.ones(n)
        for k in range(d):
            mono = mono * np.abs(W[:, k]) ** a[k]
        s += abs(c) * mono
    norm = 1.0 / math.sqrt(n) if normalize else 1.0
    return abs(weight) * norm * s


def rel_l2(a, ref):
    a = np.asarray(a, dtype=np.float64)
    ref = np.asarray(ref, dtype=np.float64)
    return float(np.linalg.norm(a - ref) / np.linalg.norm(ref))


def pde_residual(fl, ctx, dp, prob, beta):
    """Interior operator (plus the nonlinearity on block 0) of u_N minus the data at the test
    points, the derivatives from the library's FP64 evaluation of ``beta`` (a device vector)."""
    import torch
    terms = prob.blocks[0].terms
    alphas = [a for _, a in terms] + [tuple([0] * prob.d)]
    xq = torch.tensor(prob.x_test, dtype=torch.float64, device="cuda")
    ev = torch.empty((xq.shape[0], len(alphas)), dtype=torch.float64, device="cuda")
    fl.flsq_evaluate(ctx, dp.basis, beta, xq, alphas, ev)
    v = ev.cpu().numpy()
    r = v[:, :-1] @ np.array([c for c, _ in terms])
    if prob.nonlin_block == 0:
        r = r + sum(c * v[:, -1] ** k for k, c in enumerate(prob.nonlin_poly))
    return r - prob.extras["f_test"]
