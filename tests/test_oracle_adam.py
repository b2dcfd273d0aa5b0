"""Pins of the oracle's outer optimisers and of its factor-once QR.

Adam and AdamW are pinned to torch.optim.Adam / torch.optim.AdamW (an independent
implementation of Kingma and Ba's update and of Loshchilov and Hutter's decoupled
weight decay) on stand-in losses, with the same gradient function feeding both, so
only the update arithmetic is compared.  The projected variant used by the inverse
heat-source fit (w kept above a floor) is torch's Adam followed by a clamp of that
column.  The factor-once QR must reproduce the one-shot Householder solve bit for bit.
"""
import numpy as np
import pytest
import torch

import oracle
from paper_2602_10541_amd import workloads as wl


def _stand_in_grad(p):
    """A batched, non-separable smooth loss: per row h, Rosenbrock in (p0, p1) plus a quartic
    in p2 and a pull of p3 towards -0.5 (so a floor on p3 becomes active)."""
    p0, p1, p2, p3 = p[:, 0], p[:, 1], p[:, 2], p[:, 3]
    loss = (1 - p0) ** 2 + 10 * (p1 - p0 ** 2) ** 2 + (p2 - 0.3) ** 4 + 0.5 * (p3 + 0.5) ** 2 + 0.1 * p0 * p3
    g = np.stack([
        -2 * (1 - p0) - 40 * p0 * (p1 - p0 ** 2) + 0.1 * p3,
        20 * (p1 - p0 ** 2),
        4 * (p2 - 0.3) ** 3,
        (p3 + 0.5) + 0.1 * p0,
    ], axis=1)
    return loss, g


def _p0():
    rng = np.random.default_rng(4)
    return np.stack([rng.uniform(-1, 2, 8), rng.uniform(-1, 2, 8), rng.uniform(0, 1, 8),
                     rng.uniform(0.05, 0.3, 8)], axis=1)


def _torch_run(opt_cls, p0, steps, clamp=None, **kw):
    p = torch.tensor(p0, dtype=torch.float64, requires_grad=True)
    opt = opt_cls([p], **kw)
    hist = []
    for _ in range(steps):
        hist.append(p.detach().numpy().copy())
        _, g = _stand_in_grad(p.detach().numpy())
        opt.zero_grad()
        p.grad = torch.tensor(g, dtype=torch.float64)
        opt.step()
        if clamp is not None:
            with torch.no_grad():
                p[:, clamp[0]].clamp_(min=clamp[1])
    return np.array(hist), p.detach().numpy()


def _close(a, b, rtol=1e-11):
    scale = np.maximum(np.abs(b), 1e-3)
    return float(np.max(np.abs(a - b) / scale)), bool(np.all(np.abs(a - b) <= rtol * scale))


@pytest.mark.parametrize("lr", [1e-2, 5e-2])
def test_oracle_adam_matches_torch_adam(lr):
    p0 = _p0()
    hist, _, pf = oracle.adam_run(_stand_in_grad, p0, 150, lr)
    th, tf = _torch_run(torch.optim.Adam, p0, 150, lr=lr, betas=(0.9, 0.999), eps=1e-8)
    err, ok = _close(hist, th)
    assert ok, err
    err, ok = _close(pf, tf)
    assert ok, err
    # the loss fell: the stand-in is not a trivially flat run
    assert _stand_in_grad(pf)[0].sum() < 0.5 * _stand_in_grad(p0)[0].sum()


def test_oracle_projected_adam_matches_torch_adam_with_clamp():
    """The inverse fit's projection w >= 0.02 (column 3), which this loss drives into."""
    p0 = _p0()
    hist, _, pf = oracle.adam_run(_stand_in_grad, p0, 200, 1e-2, clamp_col=3, clamp_min=0.02)
    th, tf = _torch_run(torch.optim.Adam, p0, 200, clamp=(3, 0.02), lr=1e-2)
    err, ok = _close(hist, th)
    assert ok, err
    assert np.all(pf[:, 3] >= 0.02) and np.any(pf[:, 3] == 0.02)
    assert np.array_equal(pf[:, 3] == 0.02, tf[:, 3] == 0.02)


def test_oracle_adamw_matches_torch_adamw():
    p0 = _p0()
    hist, _, pf = oracle.adam_run(_stand_in_grad, p0, 120, 0.1, weight_decay=0.01)
    th, tf = _torch_run(torch.optim.AdamW, p0, 120, lr=0.1, betas=(0.9, 0.999), eps=1e-8, weight_decay=0.01)
    err, ok = _close(hist, th)
    assert ok, err
    # decoupled decay differs from L2-coupled Adam: the pin would catch the wrong variant
    hist_l2, _, _ = oracle.adam_run(lambda p: (lambda lo, g: (lo, g + 0.01 * p))(*_stand_in_grad(p)), p0, 120, 0.1)
    assert not _close(hist_l2, th)[1]


def test_oracle_adamw_sigma_matches_torch_adamw():
    def f(s):
        return (s - 7.0) ** 4 + 0.3 * s, 4.0 * (s - 7.0) ** 3 + 0.3

    sigs, losses = oracle.adamw_sigma(f, 5.0, steps=60)
    p = torch.tensor([5.0], dtype=torch.float64, requires_grad=True)
    opt = torch.optim.AdamW([p], lr=0.1, weight_decay=0.01)
    ref = []
    for _ in range(60):
        ref.append(float(p.detach()))
        opt.zero_grad()
        p.grad = torch.tensor([f(float(p.detach()))[1]], dtype=torch.float64)
        opt.step()
    assert np.allclose(sigs, ref, rtol=1e-12, atol=0)
    assert np.allclose(losses, [f(s)[0] for s in ref], rtol=1e-10)


def test_qr_factor_solve_is_the_one_shot_solve():
    rng = np.random.default_rng(8)
    prob = wl.poisson(2, 60, 3.0, 200, 40, seed=2, name="qrf", n_test=10)
    A, r = oracle.assemble_system(prob)
    Y = np.stack([r, rng.normal(size=r.shape[0]), np.zeros(r.shape[0])], axis=1)
    f = oracle.QRFactor(A, prob.mu)
    B1 = f.solve(Y)
    B2, R = oracle.tikhonov(A, Y, prob.mu, return_r=True)
    assert np.array_equal(B1, B2)
    assert np.array_equal(f.R, R)
    assert np.array_equal(f.solve(Y[:, 1]), B2[:, 1])
    # and it is the Tikhonov minimiser (LAPACK on the augmented system)
    aug = np.vstack([A, np.sqrt(prob.mu) * np.eye(A.shape[1])])
    ref = np.linalg.lstsq(aug, np.vstack([Y, np.zeros((A.shape[1], 3))]), rcond=None)[0]
    fit = A @ B1
    assert np.linalg.norm(fit - A @ ref) <= 1e-8 * np.linalg.norm(A @ ref)


def test_inverse_adam_descends_on_tiny_problem():
    prob = wl.inverse_heat(n_feat=64, sigma=3.0, n_int=300, n_ic=60, n_bc=60, n_obs=40, n_hyp=4, seed=5)
    orc0 = oracle.InverseOracle(prob, np.zeros(40))
    u_true = orc0.H @ orc0.qr.solve(orc0.rhs([wl.THETA_TRUE])[0][:, 0])
    orc = oracle.InverseOracle(prob, wl.add_noise(u_true, prob.extras["noise"]))
    hist, losses, pf = oracle.inverse_adam(orc, prob.extras["theta0"], steps=40)
    assert hist.shape == (40, 4, 4) and losses.shape == (40, 4)
    assert np.all(losses[-1] < losses[0])
    assert np.all(pf[:, 3] >= 0.02)
