"""Pins of the oracle's learnable-bandwidth functions (the reparameterisation appendix:
W_j = L What_j, outer loss ||A(L) beta*(L) - b||^2 at the regularised inner solution).

The derivative of the assembled matrix in W is checked against central differences of the
(separately pinned) assembly of Eq. (2); the loss against LAPACK's least squares on the
augmented system [A; sqrt(mu) I]; the gradient in L against central differences of that
LAPACK loss, with a regularisation weight large enough that dropping the mu terms of the
gradient fails the check; the scalar bandwidth against the trace of the L gradient.
"""
import numpy as np
import pytest

import oracle
from paper_2602_10541_amd import workloads as wl

pytestmark = pytest.mark.filterwarnings("ignore::DeprecationWarning")

TERMS = [(1.0, (2, 0, 0)), (-0.5, (0, 1, 1)), (2.0, (0, 0, 0)), (0.25, (1, 0, 3)), (-1.5, (0, 0, 1))]


@pytest.mark.parametrize("p", range(3))
def test_assemble_dW_central_differences(p):
    rng = np.random.default_rng(11 + p)
    W = rng.normal(0, 2.0, size=(7, 3))
    b = rng.uniform(0, 2 * np.pi, size=7)
    x = rng.uniform(0, 1, size=(9, 3))
    scale = rng.normal(size=7)
    h = 1e-5
    Wp, Wm = W.copy(), W.copy()
    Wp[:, p] += h * scale
    Wm[:, p] -= h * scale
    fd = (oracle.assemble(Wp, b, x, TERMS, 3.0) - oracle.assemble(Wm, b, x, TERMS, 3.0)) / (2 * h)
    got = oracle.assemble_dW(W, b, x, TERMS, p, scale, 3.0)
    assert np.abs(got - fd).max() <= 1e-7 * np.abs(fd).max()


def _small(mu):
    prob = wl.config("helmholtz_bandwidth", n_feat=40, n_int=150, n_bc=60, n_test=10)
    prob.mu = mu
    return prob


def _lapack_loss(prob, What, L):
    W = What @ np.asarray(L).T
    A = np.vstack([oracle.assemble(W, prob.b, bl.x, bl.terms, bl.weight, prob.normalize) for bl in prob.blocks])
    rhs = np.concatenate([bl.weight * bl.rhs for bl in prob.blocks])
    n = A.shape[1]
    aug = np.vstack([A, np.sqrt(prob.mu) * np.eye(n)])
    beta = np.linalg.lstsq(aug, np.concatenate([rhs, np.zeros(n)]), rcond=None)[0]
    r = A @ beta - rhs
    return float(r @ r)


def test_bandwidth_loss_matches_lapack():
    prob = _small(1e-3)
    L = np.array([[3.0, 0.0], [0.7, 2.5]])
    loss, _, beta = oracle.bandwidth_loss_and_grad(prob, prob.W, L)
    assert abs(loss - _lapack_loss(prob, prob.W, L)) <= 1e-9 * loss
    assert beta.shape == (prob.n_feat,)


@pytest.mark.parametrize("mu", [1e-3, 1e-8])
def test_bandwidth_grad_central_differences(mu):
    prob = _small(mu)
    L = np.array([[3.0, 0.0], [0.7, 2.5]])
    loss, grad, _ = oracle.bandwidth_loss_and_grad(prob, prob.W, L)
    idx = oracle.lower_index(2)
    assert len(grad) == len(idx) == 3
    h = 1e-4
    fd = []
    for p, q in idx:
        Lp, Lm = L.copy(), L.copy()
        Lp[p, q] += h
        Lm[p, q] -= h
        fd.append((_lapack_loss(prob, prob.W, Lp) - _lapack_loss(prob, prob.W, Lm)) / (2 * h))
    fd = np.array(fd)
    err = np.abs(grad - fd).max() / np.abs(fd).max()
    assert err <= 1e-5, (grad, fd)
    if mu == 1e-3:
        # the regularisation terms matter here: the gradient without them misses by far more
        W = prob.W @ L.T
        A = np.vstack([oracle.assemble(W, prob.b, bl.x, bl.terms, bl.weight) for bl in prob.blocks])
        rhs = np.concatenate([bl.weight * bl.rhs for bl in prob.blocks])
        _, _, beta = oracle.bandwidth_loss_and_grad(prob, prob.W, L)
        r = rhs - A @ beta
        naive = []
        for p, q in idx:
            dA = np.vstack([oracle.assemble_dW(W, prob.b, bl.x, bl.terms, p, prob.W[:, q], bl.weight)
                            for bl in prob.blocks])
            naive.append(-2.0 * r @ (dA @ beta))
        assert np.abs(np.array(naive) - fd).max() / np.abs(fd).max() >= 100 * max(err, 1e-7)


def test_scalar_bandwidth_is_trace_of_L_gradient():
    """W_j = sigma What_j is L = sigma I, so dLoss/dsigma = sum_p dLoss/dL_pp."""
    prob = _small(1e-6)
    sigma, h = 4.0, 1e-4
    _, grad, _ = oracle.bandwidth_loss_and_grad(prob, prob.W, sigma * np.eye(2))
    diag = [k for k, (p, q) in enumerate(oracle.lower_index(2)) if p == q]
    fd = (_lapack_loss(prob, prob.W, (sigma + h) * np.eye(2)) -
          _lapack_loss(prob, prob.W, (sigma - h) * np.eye(2))) / (2 * h)
    assert abs(grad[diag].sum() - fd) <= 1e-5 * abs(fd)


def test_bandwidth_workload_shape():
    prob = wl.config("helmholtz_bandwidth")
    assert prob.n_feat == 500 and prob.d == 2
    assert np.allclose(prob.extras["L0"], 5.0 * np.eye(2))
    # base draws at unit bandwidth
    assert abs(prob.W.std() - 1.0) < 0.08


def test_package_parameter_packing():
    """The package's packing of the scalar bandwidth and of the lower-triangular L (its AdamW runs on
    the device and is checked against the oracle's in the GPU tests); no GPU call is made."""
    from paper_2602_10541_amd.bandwidth import LearnableBandwidth, lower_pairs

    lb = LearnableBandwidth.__new__(LearnableBandwidth)
    lb.d, lb.scalar, lb.pairs = 2, True, lower_pairs(2)
    assert np.allclose(lb.L_of([2.5]), 2.5 * np.eye(2))
    lb.scalar = False
    L = np.array([[1.0, 0.0], [2.0, 3.0]])
    assert np.array_equal(lb.L_of(lb.params_of(L)), L)
