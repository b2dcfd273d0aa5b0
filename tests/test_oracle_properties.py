"""Property tests of the oracle over random dimensions, multi-indices and sizes (hypothesis).

Each property pins the oracle against something outside it: nested central differences of
sin(W . x + b) written here in numpy (Eq. (2) for |alpha| <= 4 in up to six dimensions),
linearity of the operator assembly in its terms, the agreement of the two independent C
routines (assembly times beta against the evaluation of Eq. (1)), and LAPACK's least
squares on the augmented system for random row and feature counts that are not multiples
of any tile size.
"""
import math

import numpy as np
import pytest
from hypothesis import HealthCheck, given, settings
from hypothesis import strategies as st

import oracle

SETTINGS = settings(max_examples=60, deadline=None, suppress_health_check=[HealthCheck.too_slow])


@st.composite
def multi_index(draw, max_d=6, max_order=4):
    d = draw(st.integers(1, max_d))
    order = draw(st.integers(0, max_order))
    alpha = [0] * d
    for _ in range(order):
        alpha[draw(st.integers(0, d - 1))] += 1
    return d, tuple(alpha)


def _fd_derivative(f, x, alpha, h):
    """D^alpha f at x by nested central differences (one axis at a time)."""
    if sum(alpha) == 0:
        return f(x)
    k = next(i for i, a in enumerate(alpha) if a > 0)
    lower = list(alpha)
    lower[k] -= 1
    e = np.zeros_like(x)
    e[k] = h
    return (_fd_derivative(f, x + e, tuple(lower), h) - _fd_derivative(f, x - e, tuple(lower), h)) / (2 * h)


@SETTINGS
@given(mi=multi_index(), seed=st.integers(0, 2 ** 31 - 1))
def test_assembly_is_the_derivative_of_a_feature(mi, seed):
    d, alpha = mi
    rng = np.random.default_rng(seed)
    W = rng.normal(0.0, 1.5, size=(1, d))
    b = rng.uniform(0, 2 * math.pi, size=1)
    x = rng.uniform(0, 1, size=(1, d))
    got = oracle.assemble(W, b, x, [(1.0, alpha)], normalize=False)[0, 0]
    order = sum(alpha)
    h = {0: 1.0, 1: 1e-5, 2: 1e-4, 3: 1e-3, 4: 2e-3}[order]
    fd = _fd_derivative(lambda p: math.sin(float(W[0] @ p) + b[0]), x[0], alpha, h)
    # central differences: truncation about (h^2 / 6) |W|^2 |W^alpha| per nesting level, and
    # rounding about 2^order eps / h^order
    w2 = float(np.sum(W[0] ** 2))
    bound = order * (h * h / 6.0) * w2 * max(np.max(np.abs(W[0])) ** order, 1.0) + (2 ** order) * 2e-16 / h ** order
    assert abs(got - fd) <= 4.0 * bound + 1e-15, (alpha, got, fd, bound)


@SETTINGS
@given(a1=multi_index(max_d=3), a2=multi_index(max_d=3), c1=st.floats(-3, 3), c2=st.floats(-3, 3),
       seed=st.integers(0, 2 ** 31 - 1))
def test_assembly_is_linear_in_terms(a1, a2, c1, c2, seed):
    d = max(a1[0], a2[0])
    al1 = tuple(list(a1[1]) + [0] * (d - a1[0]))
    al2 = tuple(list(a2[1]) + [0] * (d - a2[0]))
    rng = np.random.default_rng(seed)
    W = rng.normal(0.0, 2.0, size=(23, d))
    b = rng.uniform(0, 2 * math.pi, size=23)
    x = rng.uniform(0, 1, size=(17, d))
    both = oracle.assemble(W, b, x, [(c1, al1), (c2, al2)], weight=1.7)
    sep = c1 * oracle.assemble(W, b, x, [(1.0, al1)], weight=1.7) + c2 * oracle.assemble(W, b, x, [(1.0, al2)],
                                                                                        weight=1.7)
    scale = 1.7 / math.sqrt(23) * (abs(c1) + abs(c2)) * np.max(np.abs(W)) ** 4 + 1e-300
    assert np.max(np.abs(both - sep)) <= 1e-13 * scale


@SETTINGS
@given(mi=multi_index(max_d=6), n=st.integers(1, 70), q=st.integers(1, 30), seed=st.integers(0, 2 ** 31 - 1))
def test_evaluation_is_assembly_times_beta(mi, n, q, seed):
    d, alpha = mi
    rng = np.random.default_rng(seed)
    W = rng.normal(0.0, 2.0, size=(n, d))
    b = rng.uniform(0, 2 * math.pi, size=n)
    beta = rng.normal(size=n)
    x = rng.uniform(0, 1, size=(q, d))
    ev = oracle.evaluate(W, b, beta, x, [alpha])[:, 0]
    A = oracle.assemble(W, b, x, [(1.0, alpha)])
    scale = np.sum(np.abs(beta) * np.prod(np.abs(W) ** np.array(alpha)[None, :], axis=1)) / math.sqrt(n)
    assert np.max(np.abs(ev - A @ beta)) <= 1e-13 * max(scale, 1e-300)


@SETTINGS
@given(m=st.integers(3, 90), n=st.integers(1, 40), k=st.integers(1, 3), logmu=st.floats(-10, 0),
       seed=st.integers(0, 2 ** 31 - 1))
def test_tikhonov_random_shapes(m, n, k, logmu, seed):
    rng = np.random.default_rng(seed)
    A = rng.normal(size=(m, n)) * rng.uniform(0.1, 10, size=n)[None, :]
    Y = rng.normal(size=(m, k))
    mu = 10.0 ** logmu
    B = oracle.tikhonov(A, Y, mu)
    aug = np.vstack([A, math.sqrt(mu) * np.eye(n)])
    ref = np.linalg.lstsq(aug, np.vstack([Y, np.zeros((n, k))]), rcond=None)[0]
    cond = np.linalg.cond(aug)
    assert np.linalg.norm(B - ref) <= 1e-12 * cond * max(np.linalg.norm(ref), 1e-300)
    # stationarity of the Tikhonov objective: A^T (Y - A B) = mu B
    g = A.T @ (Y - A @ B) - mu * B
    assert np.linalg.norm(g) <= 1e-11 * cond * (np.linalg.norm(A) ** 2 * np.linalg.norm(B) + np.linalg.norm(A.T @ Y))
