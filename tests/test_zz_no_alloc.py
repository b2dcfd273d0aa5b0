"""The allocation-free evaluation call (static per-device scratch) against flsq_evaluate.

Both run the same kernels, so their outputs must agree bit for bit; two calls in a row, the
second smaller than the first, show that the shared scratch carries nothing from one call to
the next.  A staging size beyond the static array is refused before any work.
"""
import math

import numpy as np
import pytest

import oracle
from tests.gpu_util import context, require_gpu

pytestmark = pytest.mark.gpu


def _case(rng, d, n, n_q, sigma):
    W = rng.normal(0.0, sigma, size=(n, d))
    b = rng.uniform(0.0, 2 * math.pi, size=n)
    beta = rng.normal(size=n)
    xq = rng.uniform(0.0, 1.0, size=(n_q, d))
    return W, b, beta, xq


def _basis(fl, torch, W, b):
    Wd = torch.tensor(W, dtype=torch.float64, device="cuda")
    bd = torch.tensor(b, dtype=torch.float64, device="cuda")
    return fl.make_basis(Wd, bd, normalize=True), (Wd, bd)


@pytest.mark.parametrize("fp32", [True, False])
def test_evaluate_noalloc_matches_evaluate_twice(fp32):
    torch, fl = require_gpu()
    ctx = context()
    rng = np.random.default_rng(31)
    dt = torch.float32 if fp32 else torch.float64
    cases = [
        # heat-equation shape first (4D, N = 8192, u and its four first derivatives), then smaller
        (4, 8192, 70001, 3.0, [(0, 0, 0, 0), (1, 0, 0, 0), (0, 1, 0, 0), (0, 0, 1, 0), (0, 0, 0, 1)]),
        (2, 777, 3001, 5.0, [(0, 0), (2, 0), (1, 1)]),
    ]
    for d, n, n_q, sigma, alphas in cases:
        W, b, beta, xq = _case(rng, d, n, n_q, sigma)
        basis, keep = _basis(fl, torch, W, b)
        bt = torch.tensor(beta, dtype=torch.float64, device="cuda")
        xt = torch.tensor(xq, dtype=dt, device="cuda")
        ref = torch.full((n_q, len(alphas)), float("nan"), dtype=dt, device="cuda")
        got = torch.full((n_q, len(alphas)), float("nan"), dtype=dt, device="cuda")
        fl.flsq_evaluate(ctx, basis, bt, xt, alphas, ref)
        fl.flsq_evaluate_noalloc(ctx, basis, bt, xt, alphas, got)
        torch.cuda.synchronize()
        assert torch.isfinite(got).all()
        assert torch.equal(got, ref), (d, n, float((got - ref).abs().max()))
        # and both are the expansion of Eq. (1)-(2): the oracle on a sample of points
        idx = rng.choice(n_q, 200, replace=False)
        xs = xq[idx].astype(np.float32).astype(np.float64) if fp32 else xq[idx]
        want = oracle.evaluate(W, b, beta, xs, alphas)
        for a, al in enumerate(alphas):
            mono = np.prod(np.abs(W) ** np.array(al)[None, :], axis=1)
            scale = np.sum(np.abs(beta) * mono) / math.sqrt(n)
            err = np.abs(got[idx, a].double().cpu().numpy() - want[:, a]).max() / scale
            assert err <= (2e-5 if fp32 else 1e-13), (d, n, al, err)


def test_evaluate_noalloc_rejects_staging_beyond_scratch():
    torch, fl = require_gpu()
    ctx = context()
    rng = np.random.default_rng(5)
    d, n = 8, 40000           # 12 d N + 12 n_alpha N > 4 MiB with n_alpha = 8
    W, b, beta, xq = _case(rng, d, n, 64, 1.0)
    basis, keep = _basis(fl, torch, W, b)
    bt = torch.tensor(beta, dtype=torch.float64, device="cuda")
    xt = torch.tensor(xq, dtype=torch.float32, device="cuda")
    alphas = [tuple(1 if k == a else 0 for k in range(d)) for a in range(8)]
    out = torch.zeros((64, 8), dtype=torch.float32, device="cuda")
    with pytest.raises(fl.FlsqError) as ei:
        fl.flsq_evaluate_noalloc(ctx, basis, bt, xt, alphas, out)
    assert ei.value.status == fl.FLSQ_EINVAL
    assert "scratch" in str(ei.value)
    assert float(out.abs().max()) == 0.0
    # the allocating call takes the same size
    fl.flsq_evaluate(ctx, basis, bt, xt, alphas, out)
    assert torch.isfinite(out).all()
