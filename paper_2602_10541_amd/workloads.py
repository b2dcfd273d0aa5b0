"""Seeded synthetic workloads for the FastLSQ hot path.

This module draws inputs only: the frozen features (W, b), collocation points,
test points, and the manufactured solutions with the PDE data derived from them
by hand.  It performs none of the method's arithmetic (no assembly, no solve,
no evaluation of the random-feature expansion), so both the HIP path and the
CPU oracle can take their inputs from here.

Feature draws follow Section 2.1 / Algorithm 1 (W_j ~ N(0, sigma^2 I),
b_j ~ U(0, 2 pi)); collocation sampling follows Algorithm 1 (interior points in
the box, boundary points on its faces).  Every stream comes from
``numpy.random.SeedSequence(seed).spawn`` so each input is reproducible
independently of the others; the test set uses ``seed + 1`` (Section 3.1: test
points from a different seed).

Operators are lists of ``(coef, alpha)`` terms meaning ``sum coef * D^alpha``;
this is the linear operator of Eq. (2)/(3) written as data.
"""
from __future__ import annotations

from dataclasses import dataclass, field
import math

import numpy as np

TWO_PI = 2.0 * math.pi
PI = math.pi

# Stream order inside SeedSequence(seed).spawn(len(STREAMS)).
STREAMS = ("W", "b", "interior", "boundary", "initial", "obs", "hyp", "sweep")

# Boundary / initial-condition row weight (Section 3.1, lambda = 100).
LAM_BC = 100.0
# Tikhonov weight on ||beta||^2 (Section 2.4 / 3.1, mu = 1e-10).
MU = 1e-10


@dataclass
class Block:
    """One row block of the augmented system of Eq. (3).

    ``x`` is ``n x d`` row-major float64, ``terms`` the operator applied on these
    rows, ``weight`` multiplies both the rows and the data (lambda for boundary
    rows, 1 for interior rows), ``rhs`` is the unweighted data f or g.
    """
    name: str
    x: np.ndarray
    terms: list
    weight: float
    rhs: np.ndarray

    @property
    def n(self) -> int:
        return int(self.x.shape[0])


@dataclass
class VarBlock:
    """A row block whose operator has row-dependent coefficients:
    sum_t a_t(x_i) L_t[u](x_i), with ``channels`` = [(terms_t, a_t)] (a_t an n-array, or None
    for 1); ``weight`` and ``rhs`` as for Block."""
    name: str
    x: np.ndarray
    channels: list
    weight: float
    rhs: np.ndarray

    @property
    def n(self) -> int:
        return int(self.x.shape[0])


@dataclass
class Problem:
    name: str
    d: int
    n_feat: int
    W: np.ndarray          # n_feat x d
    b: np.ndarray          # n_feat
    blocks: list
    mu: float = MU
    normalize: bool = True
    x_test: np.ndarray | None = None
    u_test: np.ndarray | None = None
    # Pointwise nonlinearity N(u) = sum_k poly[k] u^k on block ``nonlin_block``.
    nonlin_poly: tuple | None = None
    nonlin_block: int = -1
    # First-derivative terms of the nonlinearity: sum_t c_t u^{m_t} d_{axis_t} u, as (c, m, axis).
    nonlin_adv: tuple = ()
    # Exponential term of the nonlinearity: + nonlin_exp * e^u (Bratu).
    nonlin_exp: float = 0.0
    extras: dict = field(default_factory=dict)

    @property
    def n_rows(self) -> int:
        return sum(bl.n for bl in self.blocks)


def _rngs(seed: int) -> dict:
    kids = np.random.SeedSequence(seed).spawn(len(STREAMS))
    return {name: np.random.Generator(np.random.PCG64(k)) for name, k in zip(STREAMS, kids)}


def _unit(d: int, k: int) -> tuple:
    a = [0] * d
    a[k] = 1
    return tuple(a)


def _twice(d: int, k: int) -> tuple:
    a = [0] * d
    a[k] = 2
    return tuple(a)


def laplacian_terms(d: int, dims, scale: float = 1.0) -> list:
    """``scale * sum_{k in dims} D^{2 e_k}``."""
    return [(float(scale), _twice(d, k)) for k in dims]


def identity_terms(d: int) -> list:
    return [(1.0, tuple([0] * d))]


def sample_box(rng, n: int, d: int) -> np.ndarray:
    return rng.uniform(0.0, 1.0, size=(n, d))


def sample_faces(rng, n: int, d: int, dims) -> np.ndarray:
    """Uniform points on the faces {x_k = 0} and {x_k = 1}, k in ``dims``.

    A face is drawn uniformly among the 2*len(dims) faces, then the point is
    uniform on it (faces of the unit box all have unit measure, so this is
    uniform on their union).  Coordinates outside ``dims`` stay uniform in [0,1].
    """
    dims = list(dims)
    x = rng.uniform(0.0, 1.0, size=(n, d))
    face = rng.integers(0, 2 * len(dims), size=n)
    rows = np.arange(n)
    x[rows, np.asarray(dims)[face // 2]] = (face % 2).astype(np.float64)
    return x


def draw_features(rngs, n_feat: int, sigma) -> tuple:
    sigma = np.broadcast_to(np.asarray(sigma, dtype=np.float64), (len(np.atleast_1d(sigma)),))
    d = sigma.shape[0]
    W = rngs["W"].normal(0.0, 1.0, size=(n_feat, d)) * sigma[None, :]
    b = rngs["b"].uniform(0.0, TWO_PI, size=n_feat)
    return np.ascontiguousarray(W), b


def _prod_sin(x: np.ndarray, dims) -> np.ndarray:
    out = np.ones(x.shape[0])
    for k in dims:
        out = out * np.sin(PI * x[:, k])
    return out


# ---------------------------------------------------------------------------
# The five workloads (shapes, distributions and manufactured solutions).
# ``n_feat`` / ``counts`` override the sizes for small test instances.
# ---------------------------------------------------------------------------

def poisson(d: int, n_feat: int, sigma: float, n_int: int, n_bc: int, seed: int = 0,
            name: str = "poisson", n_test: int = 5000) -> Problem:
    """-Laplace(u) = f on [0,1]^d, u = prod_k sin(pi x_k), Dirichlet data u."""
    r = _rngs(seed)
    W, b = draw_features(r, n_feat, [sigma] * d)
    xi = sample_box(r["interior"], n_int, d)
    xb = sample_faces(r["boundary"], n_bc, d, range(d))
    u = lambda x: _prod_sin(x, range(d))
    f = d * PI * PI * u(xi)
    blocks = [
        Block("interior", xi, laplacian_terms(d, range(d), -1.0), 1.0, f),
        Block("boundary", xb, identity_terms(d), LAM_BC, u(xb)),
    ]
    xt = sample_box(np.random.default_rng(seed + 1), n_test, d)
    ut = u(xt)
    return Problem(name, d, n_feat, W, b, blocks, x_test=xt, u_test=ut,
                   extras={"sigma": sigma, "exact": "prod_k sin(pi x_k)", "f_test": d * PI * PI * ut,
                           "residual_scale_test": d * PI * PI * ut})


def reaction_diffusion(n_feat: int = 2048, sigma: float = 5.0, n_int: int = 16384,
                       n_bc: int = 2048, seed: int = 0, n_test: int = 5000) -> Problem:
    """-Laplace(u) + u^3 - u = f on [0,1]^2, u = sin(2 pi x) cos(pi y).

    Laplace(u) = -5 pi^2 u, so f = 5 pi^2 u + u^3 - u.  Linear part
    L = -Laplace - I, nonlinearity N(u) = u^3 on the interior rows.
    """
    d = 2
    r = _rngs(seed)
    W, b = draw_features(r, n_feat, [sigma] * d)
    xi = sample_box(r["interior"], n_int, d)
    xb = sample_faces(r["boundary"], n_bc, d, range(d))
    u = lambda x: np.sin(2 * PI * x[:, 0]) * np.cos(PI * x[:, 1])
    ui = u(xi)
    f = 5 * PI * PI * ui + ui ** 3 - ui
    terms = laplacian_terms(d, range(d), -1.0) + [(-1.0, (0, 0))]
    blocks = [
        Block("interior", xi, terms, 1.0, f),
        Block("boundary", xb, identity_terms(d), LAM_BC, u(xb)),
    ]
    xt = sample_box(np.random.default_rng(seed + 1), n_test, d)
    ut = u(xt)
    ft = 5 * PI * PI * ut + ut ** 3 - ut
    return Problem("reaction_diffusion_2d", d, n_feat, W, b, blocks, x_test=xt, u_test=ut,
                   nonlin_poly=(0.0, 0.0, 0.0, 1.0), nonlin_block=0,
                   extras={"sigma": sigma, "exact": "sin(2 pi x) cos(pi y)", "f_test": ft,
                           "residual_scale_test": ft})


def heat(n_feat: int = 8192, sigma=(3.0, 3.0, 3.0, 1.5), n_int: int = 65536, n_ic: int = 16384,
         n_bc: int = 16384, n_query: int = 1 << 20, seed: int = 0, kappa: float = 0.1,
         n_test: int = 5000) -> Problem:
    """u_t = kappa Laplace_x u on [0,1]^3 x [0,1], coordinates (x, y, z, t).

    u = exp(-0.3 pi^2 t) prod_k sin(pi x_k) with kappa = 0.1 solves it exactly
    (u_t = -0.3 pi^2 u, Laplace_x u = -3 pi^2 u), so the interior data is 0.
    """
    d = 4
    r = _rngs(seed)
    W, b = draw_features(r, n_feat, sigma)
    xi = sample_box(r["interior"], n_int, d)
    xic = sample_box(r["initial"], n_ic, d)
    xic[:, 3] = 0.0
    xbc = sample_faces(r["boundary"], n_bc, d, range(3))
    u = lambda x: np.exp(-0.3 * PI * PI * x[:, 3]) * _prod_sin(x, range(3))
    terms = [(1.0, (0, 0, 0, 1))] + laplacian_terms(d, range(3), -kappa)
    blocks = [
        Block("interior", xi, terms, 1.0, np.zeros(n_int)),
        Block("initial", xic, identity_terms(d), LAM_BC, u(xic)),
        Block("boundary", xbc, identity_terms(d), LAM_BC, u(xbc)),
    ]
    t_rng = np.random.default_rng(seed + 1)
    xt = sample_box(t_rng, n_test, d)
    xq = None
    if n_query:
        xq = np.random.default_rng(seed + 2).uniform(0.0, 1.0, size=(n_query, d))
    ut = u(xt)
    return Problem("heat_3d_t", d, n_feat, W, b, blocks, x_test=xt, u_test=ut,
                   extras={"sigma": tuple(sigma), "kappa": kappa, "x_query": xq,
                           "exact": "exp(-0.3 pi^2 t) prod_k sin(pi x_k)", "f_test": np.zeros(n_test),
                           # u_t of the exact solution: the size of each of the two balancing terms
                           "residual_scale_test": -0.3 * PI * PI * ut})


def heat_exact_outputs(x: np.ndarray) -> np.ndarray:
    """The exact solution of the heat workload and its first derivatives at points x (n x 4):
    columns u, u_x, u_y, u_z, u_t for u = exp(-0.3 pi^2 t) prod_k sin(pi x_k)."""
    s = np.sin(PI * x[:, :3])
    c = np.cos(PI * x[:, :3])
    e = np.exp(-0.3 * PI * PI * x[:, 3])
    u = e * s[:, 0] * s[:, 1] * s[:, 2]
    ux = PI * e * c[:, 0] * s[:, 1] * s[:, 2]
    uy = PI * e * s[:, 0] * c[:, 1] * s[:, 2]
    uz = PI * e * s[:, 0] * s[:, 1] * c[:, 2]
    ut = -0.3 * PI * PI * u
    return np.stack([u, ux, uy, uz, ut], axis=1)


def gaussian_source(x: np.ndarray, theta) -> np.ndarray:
    """s(x; theta) = a exp(-|x - c|^2 / (2 w^2)) over the spatial coordinates (x, y)."""
    a, cx, cy, w = theta
    r2 = (x[:, 0] - cx) ** 2 + (x[:, 1] - cy) ** 2
    return a * np.exp(-r2 / (2.0 * w * w))


THETA_TRUE = (1.0, 0.4, 0.6, 0.1)


def inverse_heat(n_feat: int = 2048, sigma: float = 4.0, n_int: int = 8192, n_ic: int = 2048,
                 n_bc: int = 2048, n_obs: int = 400, n_hyp: int = 64, seed: int = 0,
                 kappa: float = 0.05) -> Problem:
    """u_t = kappa Laplace_x u + s(x; theta) on [0,1]^2 x [0,1], zero initial and boundary data.

    Interior operator d/dt - kappa Laplace_x; the interior data is the source
    s(x; theta), which the inverse loop replaces per hypothesis.  Coordinates
    are (x, y, t).  Observation points are uniform in space-time; the noisy
    data needs the forward solution at the true theta and is built by the
    caller with :func:`add_noise`.
    """
    d = 3
    r = _rngs(seed)
    W, b = draw_features(r, n_feat, [sigma] * d)
    xi = sample_box(r["interior"], n_int, d)
    xic = sample_box(r["initial"], n_ic, d)
    xic[:, 2] = 0.0
    xbc = sample_faces(r["boundary"], n_bc, d, range(2))
    terms = [(1.0, (0, 0, 1))] + laplacian_terms(d, range(2), -kappa)
    blocks = [
        Block("interior", xi, terms, 1.0, gaussian_source(xi, THETA_TRUE)),
        Block("initial", xic, identity_terms(d), LAM_BC, np.zeros(n_ic)),
        Block("boundary", xbc, identity_terms(d), LAM_BC, np.zeros(n_bc)),
    ]
    x_obs = sample_box(r["obs"], n_obs, d)
    hyp = r["hyp"]
    theta0 = np.stack([hyp.uniform(0.5, 1.5, n_hyp), hyp.uniform(0.2, 0.8, n_hyp),
                       hyp.uniform(0.2, 0.8, n_hyp), hyp.uniform(0.05, 0.2, n_hyp)], axis=1)
    noise = r["obs"].standard_normal(n_obs)
    return Problem("inverse_heat_2d_t", d, n_feat, W, b, blocks,
                   extras={"sigma": sigma, "kappa": kappa, "x_obs": x_obs, "theta0": theta0,
                           "theta_true": THETA_TRUE, "noise": noise})


def add_noise(u_clean: np.ndarray, noise: np.ndarray, level: float = 0.01) -> np.ndarray:
    """d_k = u_k + level * RMS(u) * xi_k (relative Gaussian noise)."""
    rms = float(np.sqrt(np.mean(u_clean ** 2)))
    return u_clean + level * rms * noise


# Named full-size workloads.
def helmholtz_sweep(n_feat: int = 1500, sigma: float = 10.0, n_int: int = 4800, n_bc: int = 1200,
                    k: float = 10.0, n_rhs: int = 64, seed: int = 0, n_test: int = 500) -> Problem:
    """Laplace u + k^2 u = 0 on [0,1]^2 with a sweep of Dirichlet data: the plane waves
    u_s = cos(k (cos t_s x + sin t_s y) + r_s), t_s and r_s uniform in [0, 2 pi), solve it
    exactly, so only the boundary rows' data change from one right-hand side to the next.

    The blocks carry u_0's data; ``extras["rhs_rows"]`` holds all n_rhs weighted right-hand
    sides (P x n_rhs, rows in block order) and ``extras["u_test_sweep"]`` the exact values at
    the test points (n_test x n_rhs).
    """
    d = 2
    r = _rngs(seed)
    W, b = draw_features(r, n_feat, [sigma] * d)
    xi = sample_box(r["interior"], n_int, d)
    xb = sample_faces(r["boundary"], n_bc, d, range(d))
    th = r["sweep"].uniform(0.0, TWO_PI, size=n_rhs)
    ph = r["sweep"].uniform(0.0, TWO_PI, size=n_rhs)

    def waves(x):
        return np.cos(k * (np.outer(x[:, 0], np.cos(th)) + np.outer(x[:, 1], np.sin(th))) + ph[None, :])

    gb = waves(xb)
    terms = laplacian_terms(d, range(d), 1.0) + [(k * k, (0, 0))]
    blocks = [
        Block("interior", xi, terms, 1.0, np.zeros(n_int)),
        Block("boundary", xb, identity_terms(d), LAM_BC, gb[:, 0].copy()),
    ]
    rhs_rows = np.concatenate([np.zeros((n_int, n_rhs)), LAM_BC * gb], axis=0)
    xt = sample_box(np.random.default_rng(seed + 1), n_test, d)
    ut = waves(xt)
    return Problem("helmholtz_2d_sweep", d, n_feat, W, b, blocks, x_test=xt, u_test=ut[:, 0].copy(),
                   extras={"sigma": sigma, "k": k, "rhs_rows": np.ascontiguousarray(rhs_rows),
                           "u_test_sweep": ut, "theta": th, "phase": ph,
                           "exact": "cos(k (cos t_s x + sin t_s y) + r_s)"})


def helmholtz_bandwidth(n_feat: int = 500, sigma0: float = 5.0, n_int: int = 2000, n_bc: int = 400,
                        k: float = 10.0, seed: int = 0, n_test: int = 500) -> Problem:
    """The learnable-bandwidth workload: Laplace u + k^2 u = f on [0,1]^2 with the exact solution
    u = sin(k x) sin(k y) (f = -k^2 u, Dirichlet data u), whose frequency k sqrt(2) lies well above
    the starting bandwidth.  ``W`` holds the frozen base draws What_j ~ N(0, I) (bandwidth 1); the
    weights used are L What_j, starting from ``extras["L0"]`` = sigma0 I."""
    d = 2
    r = _rngs(seed)
    W, b = draw_features(r, n_feat, [1.0] * d)
    xi = sample_box(r["interior"], n_int, d)
    xb = sample_faces(r["boundary"], n_bc, d, range(d))
    u = lambda x: np.sin(k * x[:, 0]) * np.sin(k * x[:, 1])
    terms = laplacian_terms(d, range(d), 1.0) + [(k * k, (0, 0))]
    blocks = [
        Block("interior", xi, terms, 1.0, -k * k * u(xi)),
        Block("boundary", xb, identity_terms(d), LAM_BC, u(xb)),
    ]
    xt = sample_box(np.random.default_rng(seed + 1), n_test, d)
    return Problem("helmholtz_2d_bandwidth", d, n_feat, W, b, blocks, x_test=xt, u_test=u(xt),
                   extras={"sigma0": sigma0, "k": k, "L0": sigma0 * np.eye(d), "exact": "sin(k x) sin(k y)"})


BURGERS_STAGES = (1.0, 0.5, 0.2, 0.1)


def burgers_1d(nu: float = 0.1, n_feat: int = 1000, sigma: float = 10.0, n_int: int = 4000, seed: int = 0,
               n_test: int = 2000) -> Problem:
    """Steady viscous Burgers u u' - nu u'' = 0 on [0, 1] with Dirichlet data from its exact
    solution u = -tanh((x - 1/2) / (2 nu)); the nonlinearity u u' acts on the interior rows.
    The continuation of Section 2.4 solves it for nu in ``BURGERS_STAGES``, each stage from the
    previous one's solution; every stage has the same features and points."""
    d = 1
    r = _rngs(seed)
    W, b = draw_features(r, n_feat, [sigma])
    xi = sample_box(r["interior"], n_int, d)
    xb = np.array([[0.0], [1.0]])
    u = lambda x: -np.tanh((x[:, 0] - 0.5) / (2.0 * nu))
    blocks = [
        VarBlock("interior", xi, [([(-nu, (2,))], None)], 1.0, np.zeros(n_int)),
        VarBlock("boundary", xb, [(identity_terms(d), None)], LAM_BC, u(xb)),
    ]
    xt = sample_box(np.random.default_rng(seed + 1), n_test, d)
    return Problem("burgers_1d", d, n_feat, W, b, blocks, x_test=xt, u_test=u(xt), nonlin_block=0,
                   nonlin_adv=((1.0, 1, 0),), extras={"sigma": sigma, "nu": nu, "exact": "-tanh((x - 1/2) / (2 nu))"})


def bratu_2d(lam: float = 1.0, n_feat: int = 1500, sigma: float = 2.0, n_int: int = 6000, n_bc: int = 1200,
             seed: int = 0, n_test: int = 5000) -> Problem:
    """Bratu -Laplace u - lambda e^u = f on [0,1]^2 (lambda = 1, sigma = 2 as in the paper's
    Newton table) with the exact solution u = sin(pi x) sin(pi y), f = 2 pi^2 u - lambda e^u, and
    zero Dirichlet data; the nonlinearity -lambda e^u acts on the interior rows."""
    d = 2
    r = _rngs(seed)
    W, b = draw_features(r, n_feat, [sigma] * d)
    xi = sample_box(r["interior"], n_int, d)
    xb = sample_faces(r["boundary"], n_bc, d, range(d))
    u = lambda x: np.sin(PI * x[:, 0]) * np.sin(PI * x[:, 1])
    f = 2 * PI * PI * u(xi) - lam * np.exp(u(xi))
    blocks = [
        VarBlock("interior", xi, [(laplacian_terms(d, range(d), -1.0), None)], 1.0, f),
        VarBlock("boundary", xb, [(identity_terms(d), None)], LAM_BC, u(xb)),
    ]
    xt = sample_box(np.random.default_rng(seed + 1), n_test, d)
    return Problem("bratu_2d", d, n_feat, W, b, blocks, x_test=xt, u_test=u(xt), nonlin_block=0, nonlin_exp=-lam,
                   extras={"sigma": sigma, "lambda": lam, "exact": "sin(pi x) sin(pi y)"})


def varcoef_2d(n_feat: int = 1500, sigma: float = 3.0, n_int: int = 6000, n_bc: int = 1200, seed: int = 0,
               n_test: int = 5000) -> Problem:
    """A coil-type operator with a variable coefficient: nu Laplace u + grad nu . grad u = g on
    [0,1]^2 with nu = 1 + sin(2 pi x) cos(pi y) / 2, exact u = sin(pi x) cos(2 pi y), g derived from
    u by hand, Dirichlet data u.  Interior channels: (Laplace, nu), (d_x, nu_x), (d_y, nu_y)."""
    d = 2
    r = _rngs(seed)
    W, b = draw_features(r, n_feat, [sigma] * d)
    xi = sample_box(r["interior"], n_int, d)
    xb = sample_faces(r["boundary"], n_bc, d, range(d))
    X, Y = xi[:, 0], xi[:, 1]
    nu = 1.0 + 0.5 * np.sin(2 * PI * X) * np.cos(PI * Y)
    nu_x = PI * np.cos(2 * PI * X) * np.cos(PI * Y)
    nu_y = -0.5 * PI * np.sin(2 * PI * X) * np.sin(PI * Y)
    u = lambda x: np.sin(PI * x[:, 0]) * np.cos(2 * PI * x[:, 1])
    ux = PI * np.cos(PI * X) * np.cos(2 * PI * Y)
    uy = -2 * PI * np.sin(PI * X) * np.sin(2 * PI * Y)
    g = nu * (-5 * PI * PI * u(xi)) + nu_x * ux + nu_y * uy
    channels = [(laplacian_terms(d, range(d), 1.0), nu), ([(1.0, (1, 0))], nu_x), ([(1.0, (0, 1))], nu_y)]
    blocks = [
        VarBlock("interior", xi, channels, 1.0, g),
        VarBlock("boundary", xb, [(identity_terms(d), None)], LAM_BC, u(xb)),
    ]
    xt = sample_box(np.random.default_rng(seed + 1), n_test, d)
    return Problem("varcoef_2d", d, n_feat, W, b, blocks, x_test=xt, u_test=u(xt),
                   extras={"sigma": sigma, "exact": "sin(pi x) cos(2 pi y)", "nu": "1 + sin(2 pi x) cos(pi y) / 2"})


def config(name: str, seed: int = 0, **kw) -> Problem:
    if name == "poisson2d":      # 2000 interior + 400 boundary, N = 500, sigma = 3, fp64
        return poisson(2, kw.pop("n_feat", 500), 3.0, kw.pop("n_int", 2000), kw.pop("n_bc", 400),
                       seed=seed, name="poisson_2d", **kw)
    if name == "poisson6d":      # 32768 interior + 8192 boundary, N = 4096, sigma = 2
        return poisson(6, kw.pop("n_feat", 4096), 2.0, kw.pop("n_int", 32768), kw.pop("n_bc", 8192),
                       seed=seed, name="poisson_6d", **kw)
    if name == "reaction2d":
        return reaction_diffusion(seed=seed, **kw)
    if name == "heat4d":
        return heat(seed=seed, **kw)
    if name == "inverse3d":
        return inverse_heat(seed=seed, **kw)
    if name == "helmholtz_sweep":   # matrix caching: 64 boundary-data sweeps, N = 1500, 6000 rows
        return helmholtz_sweep(seed=seed, **kw)
    if name == "burgers1d":             # steady Burgers, nu = 0.1 (the last continuation stage), N = 1000
        return burgers_1d(seed=seed, **kw)
    if name == "bratu2d":               # Bratu, lambda = 1, N = 1500, 7200 rows
        return bratu_2d(seed=seed, **kw)
    if name == "varcoef2d":             # coil-type variable-coefficient operator, N = 1500, 7200 rows
        return varcoef_2d(seed=seed, **kw)
    if name == "helmholtz_bandwidth":   # learnable bandwidth: N = 500 base draws, sigma0 = 5, k = 10
        return helmholtz_bandwidth(seed=seed, **kw)
    raise KeyError(name)


CONFIG_NAMES = ("poisson2d", "poisson6d", "reaction2d", "heat4d", "inverse3d")
