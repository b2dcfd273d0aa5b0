"""The manufactured data of the linear and Newton workloads at the test points, pinned by central
differences of the exact solutions written out here (independent of the generator's formulas).

The PDE residual on the test set subtracts ``extras["f_test"]`` from the interior operator of
u_N, so a wrong sign or factor there would misreport every residual."""
import math

import numpy as np
import pytest

from paper_2602_10541_amd import workloads as wl

PI = math.pi


def _fd_second(u, x, k, h=1e-4):
    e = np.zeros_like(x)
    e[:, k] = h
    return (u(x + e) - 2 * u(x) + u(x - e)) / (h * h)


def _fd_first(u, x, k, h=1e-5):
    e = np.zeros_like(x)
    e[:, k] = h
    return (u(x + e) - u(x - e)) / (2 * h)


@pytest.mark.parametrize("d", [2, 6])
def test_poisson_f_test_is_minus_laplacian(d):
    prob = wl.poisson(d, 16, 2.0, 10, 10, seed=3, n_test=50)
    u = lambda x: np.prod(np.sin(PI * x), axis=1)
    x = prob.x_test
    lap = sum(_fd_second(u, x, k) for k in range(d))
    np.testing.assert_allclose(prob.extras["f_test"], -lap, rtol=1e-5, atol=1e-5)
    np.testing.assert_allclose(prob.u_test, u(x), rtol=0, atol=1e-15)


def test_reaction_f_test():
    prob = wl.reaction_diffusion(n_feat=16, n_int=10, n_bc=10, seed=2, n_test=50)
    u = lambda x: np.sin(2 * PI * x[:, 0]) * np.cos(PI * x[:, 1])
    x = prob.x_test
    lap = _fd_second(u, x, 0) + _fd_second(u, x, 1)
    ux = u(x)
    np.testing.assert_allclose(prob.extras["f_test"], -lap + ux ** 3 - ux, rtol=1e-5, atol=1e-5)


def test_heat_f_test_and_scale():
    prob = wl.heat(n_feat=16, n_int=10, n_ic=10, n_bc=10, n_query=0, seed=2, n_test=50)
    u = lambda x: np.exp(-0.3 * PI * PI * x[:, 3]) * np.prod(np.sin(PI * x[:, :3]), axis=1)
    x = prob.x_test
    ut = _fd_first(u, x, 3)
    lap = sum(_fd_second(u, x, k) for k in range(3))
    # the operator d/dt - 0.1 Laplace_x annihilates the exact solution, and the scale is its u_t
    np.testing.assert_allclose(ut - 0.1 * lap, prob.extras["f_test"], atol=1e-5)
    np.testing.assert_allclose(prob.extras["residual_scale_test"], ut, rtol=1e-6, atol=1e-8)


def test_heat_exact_outputs_are_u_and_its_gradient():
    u = lambda x: np.exp(-0.3 * PI * PI * x[:, 3]) * np.prod(np.sin(PI * x[:, :3]), axis=1)
    x = np.random.default_rng(4).uniform(0, 1, size=(40, 4))
    ex = wl.heat_exact_outputs(x)
    np.testing.assert_allclose(ex[:, 0], u(x), rtol=0, atol=1e-15)
    for k in range(4):
        np.testing.assert_allclose(ex[:, 1 + k], _fd_first(u, x, k), rtol=1e-7, atol=1e-8)
