"""Pins of the CPU oracle against facts fixed by the paper and by mathematics.

Each test checks the oracle against something other than itself: symbolic
derivatives evaluated at 30 digits, finite differences, the closed forms of
Corollary 2.1, the phase-shift identity of Appendix F, LAPACK's SVD-based least
squares, an mpmath solve of the normal equations, exact interpolation, and
statistics of the feature draw.  A dropped term, a wrong sign or index, or a
transposed operand in the oracle fails at least one of them.
"""
import math

import mpmath
import numpy as np
import pytest
import sympy as sp

import oracle
from paper_2602_10541_amd import workloads as wl

pytestmark = pytest.mark.filterwarnings("ignore::DeprecationWarning")


def _rand_feature(rng, d, scale=3.0):
    W = rng.normal(0, scale, size=(1, d))
    b = rng.uniform(0, 2 * math.pi, size=1)
    return W, b


# ---------------------------------------------------------------- Eq. (2) assembly

@pytest.mark.parametrize("seed", range(6))
def test_assembly_matches_symbolic_derivative(seed):
    """D^alpha sin(W.x + b) from sympy at rational points, 30 digits, vs the oracle."""
    rng = np.random.default_rng(100 + seed)
    d = int(rng.integers(1, 5))
    xs = sp.symbols(f"x0:{d}")
    # rational W, b, x so the symbolic value is exact before evaluation
    Wq = [sp.Rational(int(rng.integers(-40, 41)), 10) for _ in range(d)]
    bq = sp.Rational(int(rng.integers(0, 63)), 10)
    xq = [sp.Rational(int(rng.integers(0, 101)), 100) for _ in range(d)]
    phi = sp.sin(sum(w * x for w, x in zip(Wq, xs)) + bq)
    W = np.array([[float(w) for w in Wq]])
    b = np.array([float(bq)])
    x = np.array([[float(v) for v in xq]])
    for _ in range(6):
        alpha = tuple(int(a) for a in rng.integers(0, 3, size=d))
        if sum(alpha) > 4:
            continue
        expr = phi
        for k, a in enumerate(alpha):
            if a:
                expr = sp.diff(expr, xs[k], a)
        exact = sp.N(expr.subs(dict(zip(xs, xq))), 30)
        got = oracle.assemble(W, b, x, [(1.0, alpha)], weight=1.0, normalize=False)[0, 0]
        mono = float(np.prod(np.abs(W[0]) ** np.array(alpha))) or 1.0
        assert abs(got - float(exact)) <= 1e-13 * max(1.0, mono), (alpha, got, exact)


def test_assembly_central_differences():
    """First and second derivatives of one feature against central differences."""
    rng = np.random.default_rng(7)
    d = 3
    W, b = _rand_feature(rng, d, 2.0)
    x = rng.uniform(0, 1, size=(1, d))
    h1, h2 = 1e-5, 1e-4
    f = lambda xx: oracle.assemble(W, b, xx, [(1.0, (0,) * d)], normalize=False)[0, 0]
    for k in range(d):
        e = np.zeros((1, d))
        e[0, k] = 1.0
        a1 = tuple(1 if i == k else 0 for i in range(d))
        a2 = tuple(2 if i == k else 0 for i in range(d))
        fd1 = (f(x + h1 * e) - f(x - h1 * e)) / (2 * h1)
        fd2 = (f(x + h2 * e) - 2 * f(x) + f(x - h2 * e)) / (h2 * h2)
        g1 = oracle.assemble(W, b, x, [(1.0, a1)], normalize=False)[0, 0]
        g2 = oracle.assemble(W, b, x, [(1.0, a2)], normalize=False)[0, 0]
        assert abs(g1 - fd1) < 1e-8 * max(1, abs(W[0, k]))
        assert abs(g2 - fd2) < 1e-5 * max(1, W[0, k] ** 2)


def test_corollary_common_operators():
    """Laplacian, biharmonic and advection closed forms of Corollary 2.1."""
    rng = np.random.default_rng(11)
    d = 4
    N = 7
    W = rng.normal(0, 2.5, size=(N, d))
    b = rng.uniform(0, 2 * math.pi, N)
    x = rng.uniform(0, 1, size=(5, d))
    z = x @ W.T + b
    nW2 = np.sum(W ** 2, axis=1)
    lap = wl.laplacian_terms(d, range(d), 1.0)
    A_lap = oracle.assemble(W, b, x, lap, normalize=False)
    np.testing.assert_allclose(A_lap, -nW2[None, :] * np.sin(z), rtol=0, atol=1e-12 * nW2.max())
    bih = []
    for k in range(d):
        for l in range(d):
            a = [0] * d
            a[k] += 2
            a[l] += 2
            bih.append((1.0, tuple(a)))
    A_bih = oracle.assemble(W, b, x, bih, normalize=False)
    np.testing.assert_allclose(A_bih, (nW2 ** 2)[None, :] * np.sin(z), rtol=0, atol=1e-11 * (nW2 ** 2).max())
    v = rng.normal(size=d)
    adv = [(float(v[k]), tuple(1 if i == k else 0 for i in range(d))) for k in range(d)]
    A_adv = oracle.assemble(W, b, x, adv, normalize=False)
    np.testing.assert_allclose(A_adv, (W @ v)[None, :] * np.cos(z), rtol=0, atol=1e-12 * np.abs(W @ v).max())


def test_fourth_order_returns_plus_sin_and_phase_shift():
    """|alpha| = 4 cycles back to +sin; D^{e_k} phi(b) = W_k phi(b + pi/2) (Appendix F shift)."""
    rng = np.random.default_rng(3)
    d = 2
    W = rng.normal(0, 2, size=(3, d))
    b = rng.uniform(0, 2 * math.pi, 3)
    x = rng.uniform(0, 1, size=(4, d))
    z = x @ W.T + b
    A4 = oracle.assemble(W, b, x, [(1.0, (4, 0))], normalize=False)
    np.testing.assert_allclose(A4, W[:, 0] ** 4 * np.sin(z), atol=1e-12 * (W[:, 0] ** 4).max())
    A31 = oracle.assemble(W, b, x, [(1.0, (3, 1))], normalize=False)
    np.testing.assert_allclose(A31, W[:, 0] ** 3 * W[:, 1] * np.sin(z), atol=1e-11)
    A1 = oracle.assemble(W, b, x, [(1.0, (0, 1))], normalize=False)
    A0s = oracle.assemble(W, b + math.pi / 2, x, [(1.0, (0, 0))], normalize=False)
    np.testing.assert_allclose(A1, W[:, 1][None, :] * A0s, atol=1e-13 * np.abs(W).max())


def test_weight_and_normalisation():
    """Eq. (3) row weight and the 1/sqrt(N) of Eq. (1) scale every entry."""
    rng = np.random.default_rng(5)
    W = rng.normal(0, 1, size=(16, 2))
    b = rng.uniform(0, 6, 16)
    x = rng.uniform(0, 1, size=(3, 2))
    A1 = oracle.assemble(W, b, x, [(1.0, (0, 0))], weight=1.0, normalize=False)
    A2 = oracle.assemble(W, b, x, [(1.0, (0, 0))], weight=100.0, normalize=True)
    np.testing.assert_allclose(A2, 100.0 / 4.0 * A1, rtol=1e-15)
    np.testing.assert_allclose(A1, np.sin(x @ W.T + b), atol=1e-15)


# ---------------------------------------------------------------- Tikhonov solve

def test_tikhonov_matches_lapack_svd_lstsq():
    rng = np.random.default_rng(21)
    A = rng.normal(size=(60, 25))
    A[:, 3] = A[:, 4] + 1e-6 * rng.normal(size=60)          # near-dependent columns
    r = rng.normal(size=60)
    mu = 1e-4
    beta = oracle.tikhonov(A, r, mu)
    Aug = np.vstack([A, math.sqrt(mu) * np.eye(25)])
    ref = np.linalg.lstsq(Aug, np.concatenate([r, np.zeros(25)]), rcond=None)[0]
    np.testing.assert_allclose(beta, ref, rtol=1e-9, atol=1e-9)


def test_tikhonov_kkt_and_multi_rhs():
    """A^T (rhs - A beta) = mu beta for each right-hand side column."""
    rng = np.random.default_rng(22)
    A = rng.normal(size=(80, 30))
    Y = rng.normal(size=(80, 3))
    mu = 1e-3
    B = oracle.tikhonov(A, Y, mu)
    for c in range(3):
        g = A.T @ (Y[:, c] - A @ B[:, c])
        np.testing.assert_allclose(g, mu * B[:, c], atol=1e-11)
        np.testing.assert_allclose(B[:, c], oracle.tikhonov(A, Y[:, c], mu), rtol=1e-12)


def test_tikhonov_against_mpmath_normal_equations():
    rng = np.random.default_rng(23)
    m, n = 18, 7
    A = rng.normal(size=(m, n))
    r = rng.normal(size=m)
    mu = 1e-6
    mpmath.mp.dps = 50
    Am = mpmath.matrix(A.tolist())
    G = Am.T * Am + mu * mpmath.eye(n)
    c = Am.T * mpmath.matrix(r.tolist())
    ref = np.array([float(v) for v in mpmath.lu_solve(G, c)])
    beta = oracle.tikhonov(A, r, mu)
    np.testing.assert_allclose(beta, ref, rtol=1e-12, atol=1e-13)


def test_tikhonov_square_interpolates():
    """Square, well-conditioned, mu = 0: the solve interpolates A beta = rhs."""
    rng = np.random.default_rng(24)
    A = rng.normal(size=(12, 12)) + 6 * np.eye(12)
    r = rng.normal(size=12)
    beta = oracle.tikhonov(A, r, 0.0)
    np.testing.assert_allclose(A @ beta, r, atol=1e-13)
    np.testing.assert_allclose(beta, np.linalg.solve(A, r), rtol=1e-12)


def test_r_factor_and_trisolve():
    """R^T R = A^T A + mu I; trisolve inverts R and R^T."""
    rng = np.random.default_rng(25)
    A = rng.normal(size=(40, 9))
    mu = 1e-2
    _, R = oracle.tikhonov(A, np.zeros(40), mu, return_r=True)
    np.testing.assert_allclose(R.T @ R, A.T @ A + mu * np.eye(9), atol=1e-11)
    y = rng.normal(size=(9, 2))
    np.testing.assert_allclose(R @ oracle.trisolve(R, y), y, atol=1e-12)
    np.testing.assert_allclose(R.T @ oracle.trisolve(R, y, transpose=True), y, atol=1e-12)


# ---------------------------------------------------------------- evaluation

def test_evaluate_symbolic_and_fd():
    rng = np.random.default_rng(31)
    d, N = 2, 5
    Wq = [[sp.Rational(int(rng.integers(-30, 31)), 10) for _ in range(d)] for _ in range(N)]
    bq = [sp.Rational(int(rng.integers(0, 63)), 10) for _ in range(N)]
    betaq = [sp.Rational(int(rng.integers(-9, 10)), 7) for _ in range(N)]
    xs = sp.symbols("x0:2")
    u = sum(bt * sp.sin(sum(w * x for w, x in zip(Wj, xs)) + bj) for bt, Wj, bj in zip(betaq, Wq, bq))
    u = u / sp.sqrt(N)
    pt = [sp.Rational(3, 10), sp.Rational(7, 10)]
    W = np.array([[float(v) for v in r] for r in Wq])
    b = np.array([float(v) for v in bq])
    beta = np.array([float(v) for v in betaq])
    alphas = [(0, 0), (1, 0), (0, 1), (2, 0), (1, 1), (0, 3)]
    got = oracle.evaluate(W, b, beta, np.array([[0.3, 0.7]]), alphas)[0]
    for a, g in zip(alphas, got):
        e = u
        for k, n in enumerate(a):
            if n:
                e = sp.diff(e, xs[k], n)
        exact = float(sp.N(e.subs(dict(zip(xs, pt))), 30))
        assert abs(g - exact) < 1e-12 * max(1.0, abs(exact)), (a, g, exact)


# ---------------------------------------------------------------- linear solve on a workload

def test_linear_poisson_manufactured_band():
    """Algorithm 1 on the 2D Poisson workload: error band vs the exact solution (band only)."""
    prob = wl.config("poisson2d")
    beta = oracle.solve_linear(prob)
    u = oracle.evaluate(prob.W, prob.b, beta, prob.x_test, [(0, 0)])[:, 0]
    err = oracle.rel_l2(u, prob.u_test)
    assert err < 1e-6, err
    A, r = oracle.assemble_system(prob)
    g = A.T @ (r - A @ beta)
    assert np.linalg.norm(g - prob.mu * beta) < 1e-6 * np.linalg.norm(A.T @ r)


def test_helmholtz_sweep_manufactured_and_columns():
    """The sweep's plane waves solve Laplace u + k^2 u = 0 (central differences), its boundary
    data are the waves on the faces, and one multi-right-hand-side oracle solve gives each
    column's single solve and a small error against the exact waves (band only)."""
    prob = wl.helmholtz_sweep(n_feat=300, n_int=1200, n_bc=300, n_rhs=4, seed=2, n_test=400)
    k, th, ph = prob.extras["k"], prob.extras["theta"], prob.extras["phase"]
    wave = lambda x, y, s: np.cos(k * (math.cos(th[s]) * x + math.sin(th[s]) * y) + ph[s])
    rng = np.random.default_rng(0)
    h = 1e-4
    for s in range(4):
        x, y = rng.uniform(0.1, 0.9, 2)
        lap = (wave(x + h, y, s) + wave(x - h, y, s) + wave(x, y + h, s) + wave(x, y - h, s) - 4 * wave(x, y, s)) / h**2
        assert abs(lap + k * k * wave(x, y, s)) < 1e-4 * k * k
    xb = prob.blocks[1].x
    Y = prob.extras["rhs_rows"]
    assert np.all(np.isclose(np.min(np.minimum(xb, 1 - xb), axis=1), 0.0))
    for s in range(4):
        np.testing.assert_allclose(Y[prob.blocks[0].n:, s], wl.LAM_BC * wave(xb[:, 0], xb[:, 1], s), rtol=0, atol=1e-12)
        assert np.all(Y[:prob.blocks[0].n, s] == 0.0)
    A, _ = oracle.assemble_system(prob)
    B = oracle.tikhonov(A, Y, prob.mu)
    for s in range(4):
        np.testing.assert_allclose(B[:, s], oracle.tikhonov(A, Y[:, s], prob.mu), rtol=1e-9, atol=1e-9 * np.abs(B[:, s]).max())
        u = oracle.evaluate(prob.W, prob.b, B[:, s], prob.x_test, [(0, 0)])[:, 0]
        assert oracle.rel_l2(u, prob.extras["u_test_sweep"][:, s]) < 1e-4


# ---------------------------------------------------------------- Newton

def _tiny_reaction(n_feat=300, n_int=900, n_bc=200, sigma=4.0):
    return wl.reaction_diffusion(n_feat=n_feat, sigma=sigma, n_int=n_int, n_bc=n_bc, seed=3, n_test=500)


def test_newton_descends_and_matches_scipy_least_squares():
    """Gauss-Newton with Tikhonov steps (Eq. (4)-(5)) against scipy's Levenberg-Marquardt.

    scipy minimises ||R(beta)||^2 + mu ||beta||^2 with its own algorithm; after
    the fast phase both land on the same solution u to within the slow plateau
    drift the paper describes (Appendix C).  The residual norm must fall at every
    accepted step (Armijo) and by two orders in the first step.
    """
    from scipy.optimize import least_squares
    prob = _tiny_reaction()
    beta, trace = oracle.solve_newton(prob, max_iter=15)
    norms = [t["res_norm"] for t in trace]
    assert all(b < a for a, b in zip(norms, norms[1:]))
    assert norms[1] < 1e-2 * norms[0]
    mu = prob.mu

    def fun(bt):
        r, _ = oracle.newton_residual(prob, bt)
        return np.concatenate([r, math.sqrt(mu) * bt])

    def jac(bt):
        _, us = oracle.newton_residual(prob, bt)
        return np.vstack([oracle.newton_jacobian(prob, us), math.sqrt(mu) * np.eye(len(bt))])

    sol = least_squares(fun, oracle.solve_linear(prob), jac=jac, method="lm", xtol=1e-15, ftol=1e-15,
                        gtol=1e-15, max_nfev=200)
    u_ref = oracle.evaluate(prob.W, prob.b, sol.x, prob.x_test, [(0, 0)])[:, 0]
    u_got = oracle.evaluate(prob.W, prob.b, beta, prob.x_test, [(0, 0)])[:, 0]
    assert oracle.rel_l2(u_got, u_ref) < 2e-6
    assert oracle.rel_l2(u_got, prob.u_test) < 2e-6


def test_newton_jacobian_central_differences():
    """J = dR/dbeta (Section 2.4) against central differences of the residual."""
    prob = _tiny_reaction(n_feat=12, n_int=30, n_bc=10, sigma=2.0)
    rng = np.random.default_rng(1)
    beta = rng.normal(size=12)
    _, us = oracle.newton_residual(prob, beta)
    J = oracle.newton_jacobian(prob, us)
    h = 1e-6
    for j in (0, 5, 11):
        e = np.zeros(12)
        e[j] = h
        fd = (oracle.newton_residual(prob, beta + e)[0] - oracle.newton_residual(prob, beta - e)[0]) / (2 * h)
        np.testing.assert_allclose(J[:, j], fd, rtol=1e-6, atol=1e-6 * np.abs(fd).max())


# ---------------------------------------------------------------- adjoint

def _tiny_inverse():
    prob = wl.inverse_heat(n_feat=64, sigma=3.0, n_int=300, n_ic=60, n_bc=60, n_obs=40, n_hyp=4, seed=5)
    orc0 = oracle.InverseOracle(prob, np.zeros(40))
    u_true = orc0.H @ oracle.tikhonov(orc0.A, orc0.rhs([wl.THETA_TRUE])[0][:, 0], prob.mu)
    data = wl.add_noise(u_true, prob.extras["noise"])
    return prob, oracle.InverseOracle(prob, data)


def test_adjoint_gradient_central_differences():
    prob, orc = _tiny_inverse()
    thetas = prob.extras["theta0"]
    loss, g, gk, _ = orc.loss_and_grad(thetas)
    h = 1e-6
    for hyp in range(2):
        for p in range(4):
            tp = thetas[hyp].copy()
            tm = thetas[hyp].copy()
            step = h * max(1.0, abs(tp[p]))
            tp[p] += step
            tm[p] -= step
            fd = (orc.loss([tp])[0] - orc.loss([tm])[0]) / (2 * step)
            assert abs(g[hyp, p] - fd) <= 1e-5 * max(abs(fd), 1e-3 * np.abs(g[hyp]).max()), (hyp, p, g[hyp, p], fd)
    k0 = orc.kappa
    hk = 1e-6
    fdk = (orc.loss(thetas[:1], kappa=k0 + hk)[0] - orc.loss(thetas[:1], kappa=k0 - hk)[0]) / (2 * hk)
    assert abs(gk[0] - fdk) <= 1e-5 * abs(fdk), (gk[0], fdk)


def test_adjoint_amplitude_closed_form():
    """rhs is linear in a, so u_obs = a h1 and dL/da = (2/n) sum (a h1 - d) h1 exactly."""
    prob, orc = _tiny_inverse()
    th = np.array(prob.extras["theta0"][0])
    th1 = th.copy()
    th1[0] = 1.0
    Rhs1, _ = orc.rhs([th1])
    h1 = orc.H @ oracle.tikhonov(orc.A, Rhs1[:, 0], prob.mu)
    a = th[0]
    n = h1.shape[0]
    exact = (2.0 / n) * np.sum((a * h1 - orc.data) * h1)
    _, g, _, _ = orc.loss_and_grad(th[None, :])
    assert abs(g[0, 0] - exact) <= 1e-10 * abs(exact)


# ---------------------------------------------------------------- feature draw statistics

def test_kernel_limit_has_half_factor():
    """(1/N) sum_j phi_j(x) phi_j(x') -> 0.5 exp(-sigma^2 |x - x'|^2 / 2) for uniform phases."""
    N, sigma = 200000, 2.0
    rngs = wl._rngs(9)
    W, b = wl.draw_features(rngs, N, [sigma, sigma])
    x = np.array([[0.2, 0.3], [0.25, 0.45], [0.9, 0.1]])
    H = oracle.assemble(W, b, x, [(1.0, (0, 0))], normalize=False)
    K = H @ H.T / N
    for i in range(3):
        for j in range(3):
            ref = 0.5 * math.exp(-sigma ** 2 * np.sum((x[i] - x[j]) ** 2) / 2)
            assert abs(K[i, j] - ref) < 5.0 / math.sqrt(N), (i, j, K[i, j], ref)
    assert abs(W.std() - sigma) < 0.02 and abs(b.mean() - math.pi) < 0.03


def test_device_sine_polynomial_constants():
    """The FP64 sine polynomial in csrc/flsq_device.h (sin_poly, used by sin_f64), read from the header and
    evaluated in double as the kernel does (Horner in r^2, then r + (r r^2) p): within 2.5e-16
    of math.sin on the reduced interval [-pi/2, pi/2]; its two lowest coefficients are the
    Taylor ones to rounding (-1/3!, 1/5!), as a fit of (sin r - r) / r^3 must give."""
    import math
    import re
    from pathlib import Path
    src = (Path(__file__).resolve().parents[1] / "paper_2602_10541_amd" / "csrc" / "flsq_device.h").read_text()
    body = src[src.index("SinPoly sin_poly()"):src.index("SinPoly sin_poly_sgpr()")]
    coef = [float(m) for m in re.findall(r"(-?[0-9]+\.[0-9]+(?:e-?[0-9]+)?)", body)]
    assert len(coef) == 8, coef
    assert abs(coef[-1] + 1 / 6) < 1e-16 and abs(coef[-2] - 1 / 120) < 1e-15
    worst = 0.0
    for i in range(-4000, 4001):
        r = (math.pi / 2) * i / 4000
        r2 = r * r
        p = coef[0]
        for c in coef[1:]:
            p = math.fma(p, r2, c) if hasattr(math, "fma") else p * r2 + c
        s = r + (r * r2) * p
        worst = max(worst, abs(s - math.sin(r)))
    assert worst <= 2.5e-16, worst
