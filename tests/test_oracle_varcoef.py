"""Pins of the oracle's row-dependent-coefficient operators and first-derivative nonlinearities.

- The coil-type operator nu Laplace u + grad nu . grad u, assembled from three channels, is the
  divergence of the flux nu grad u: checked against central differences of that flux, built
  from the separately pinned evaluation of Eq. (1)-(2).
- The workloads' data: the tanh profile solves steady Burgers exactly and the variable-
  coefficient source matches its exact solution (sympy, symbolic).
- The linear solve against LAPACK least squares on [A; sqrt(mu) I].
- The Newton Jacobian with the u u' term against central differences of the residual, and the
  Newton solution against scipy's Levenberg-Marquardt on the same regularised residual.
- Continuation reaches the exact Burgers solution within a band on a small instance.
- The Bratu exponential term: its Jacobian against central differences and its data (sympy).
"""
import math

import numpy as np
import pytest
import sympy as sp

import oracle
from paper_2602_10541_amd import workloads as wl

pytestmark = pytest.mark.filterwarnings("ignore::DeprecationWarning")


def test_varcoef_operator_is_divergence_of_flux():
    prob = wl.varcoef_2d(n_feat=60, n_int=40, n_bc=10, n_test=10)
    rng = np.random.default_rng(5)
    beta = rng.normal(size=prob.n_feat)
    bl = prob.blocks[0]
    A = oracle.assemble_var(prob.W, prob.b, bl.x, bl.channels, bl.weight, prob.normalize)

    def nu(x):
        return 1.0 + 0.5 * np.sin(2 * np.pi * x[:, 0]) * np.cos(np.pi * x[:, 1])

    def flux(x, k):
        g = oracle.evaluate(prob.W, prob.b, beta, x, [(1, 0), (0, 1)])
        return nu(x) * g[:, k]

    h = 1e-5
    div = np.zeros(bl.n)
    for k in range(2):
        e = np.zeros(2)
        e[k] = h
        div += (flux(bl.x + e, k) - flux(bl.x - e, k)) / (2 * h)
    got = A @ beta
    assert np.abs(got - div).max() <= 1e-6 * np.abs(div).max()
    # a channel whose coefficient is None is the constant-coefficient assembly
    Ab = oracle.assemble_var(prob.W, prob.b, bl.x, [(wl.laplacian_terms(2, range(2)), None)])
    assert np.array_equal(Ab, oracle.assemble(prob.W, prob.b, bl.x, wl.laplacian_terms(2, range(2))))


def test_workload_data_symbolic():
    x, y, nu = sp.symbols("x y nu", real=True)
    u = -sp.tanh((x - sp.Rational(1, 2)) / (2 * nu))
    assert sp.simplify(u * sp.diff(u, x) - nu * sp.diff(u, x, 2)) == 0
    N = 1 + sp.sin(2 * sp.pi * x) * sp.cos(sp.pi * y) / 2
    U = sp.sin(sp.pi * x) * sp.cos(2 * sp.pi * y)
    g = sp.diff(N * sp.diff(U, x), x) + sp.diff(N * sp.diff(U, y), y)
    prob = wl.varcoef_2d(n_feat=10, n_int=25, n_bc=4, n_test=4)
    f = sp.lambdify((x, y), g, "numpy")
    bl = prob.blocks[0]
    assert np.abs(f(bl.x[:, 0], bl.x[:, 1]) - bl.rhs).max() <= 1e-12 * np.abs(bl.rhs).max()
    b = wl.burgers_1d(nu=0.2, n_feat=10, n_int=10, n_test=10)
    ub = sp.lambdify(x, u.subs(nu, 0.2), "numpy")
    assert np.allclose(b.blocks[1].rhs, ub(b.blocks[1].x[:, 0]), rtol=0, atol=1e-15)


def test_linear_var_matches_lapack():
    prob = wl.varcoef_2d(n_feat=80, n_int=300, n_bc=80, n_test=10)
    prob.mu = 1e-8
    beta = oracle.solve_linear_var(prob)
    A, r = oracle.assemble_var_system(prob)
    n = A.shape[1]
    ref = np.linalg.lstsq(np.vstack([A, math.sqrt(prob.mu) * np.eye(n)]), np.concatenate([r, np.zeros(n)]),
                          rcond=None)[0]
    assert np.linalg.norm(A @ (beta - ref)) <= 1e-9 * np.linalg.norm(r)


def _tiny_burgers(nu=0.5):
    return wl.burgers_1d(nu=nu, n_feat=40, sigma=4.0, n_int=120, n_test=200)


def test_burgers_jacobian_central_differences():
    prob = _tiny_burgers()
    rng = np.random.default_rng(2)
    beta = oracle.solve_linear_var(prob) + 0.1 * rng.normal(size=prob.n_feat)
    J = oracle.newton_var_jacobian(prob, beta)
    v = rng.normal(size=prob.n_feat)
    h = 1e-6
    fd = (oracle.newton_var_residual(prob, beta + h * v)[0] - oracle.newton_var_residual(prob, beta - h * v)[0]) / (2 * h)
    assert np.abs(J @ v - fd).max() <= 1e-6 * np.abs(fd).max()
    # without the u' dN/d(u') part the Jacobian misses by far more
    zero = (0,)
    bl = prob.blocks[0]
    ev = oracle.evaluate(prob.W, prob.b, beta, bl.x, [zero, (1,)])
    Jbad = J.copy()
    Jbad[:bl.n] -= ev[:, 0][:, None] * oracle.assemble(prob.W, prob.b, bl.x, [(1.0, (1,))], bl.weight)
    assert np.abs(Jbad @ v - fd).max() >= 1e-2 * np.abs(fd).max()


def test_burgers_newton_matches_scipy_least_squares():
    from scipy.optimize import least_squares
    prob = _tiny_burgers()
    beta, trace = oracle.solve_newton_var(prob, max_iter=20, tol_du=1e-12)
    norms = [t["res_norm"] for t in trace]
    assert norms[1] < 1e-2 * norms[0]
    mu = prob.mu

    def fun(bt):
        return np.concatenate([oracle.newton_var_residual(prob, bt)[0], math.sqrt(mu) * bt])

    sol = least_squares(fun, oracle.solve_linear_var(prob), method="lm", xtol=1e-15, ftol=1e-15, gtol=1e-15,
                        max_nfev=4000)
    u_ref = oracle.evaluate(prob.W, prob.b, sol.x, prob.x_test, [(0,)])[:, 0]
    u_got = oracle.evaluate(prob.W, prob.b, beta, prob.x_test, [(0,)])[:, 0]
    assert oracle.rel_l2(u_got, u_ref) < 1e-6
    assert oracle.rel_l2(u_got, prob.u_test) < 1e-4


def test_burgers_continuation_band():
    """Four-stage continuation (nu = 1, 0.5, 0.2, 0.1) on a small instance ends near the exact
    tanh profile; every stage after the first starts from the previous solution."""
    beta, traces = oracle.continuation(
        lambda nu: wl.burgers_1d(nu=nu, n_feat=200, n_int=800, n_test=500), wl.BURGERS_STAGES, max_iter=20,
        tol_du=1e-8)
    assert len(traces) == 4
    prob = wl.burgers_1d(nu=0.1, n_feat=200, n_int=800, n_test=500)
    u = oracle.evaluate(prob.W, prob.b, beta, prob.x_test, [(0,)])[:, 0]
    assert oracle.rel_l2(u, prob.u_test) < 3e-4   # 8e-5 at N = 200


def test_bratu_jacobian_and_data():
    prob = wl.bratu_2d(n_feat=50, n_int=120, n_bc=40, n_test=10)
    x, y = sp.symbols("x y", real=True)
    U = sp.sin(sp.pi * x) * sp.sin(sp.pi * y)
    f = sp.lambdify((x, y), -sp.diff(U, x, 2) - sp.diff(U, y, 2) - sp.exp(U), "numpy")
    bl = prob.blocks[0]
    assert np.abs(f(bl.x[:, 0], bl.x[:, 1]) - bl.rhs).max() <= 1e-12 * np.abs(bl.rhs).max()
    rng = np.random.default_rng(4)
    beta = oracle.solve_linear_var(prob) + 0.05 * rng.normal(size=prob.n_feat)
    J = oracle.newton_var_jacobian(prob, beta)
    v = rng.normal(size=prob.n_feat)
    h = 1e-6
    fd = (oracle.newton_var_residual(prob, beta + h * v)[0] - oracle.newton_var_residual(prob, beta - h * v)[0]) / (2 * h)
    assert np.abs(J @ v - fd).max() <= 1e-6 * np.abs(fd).max()
