"""Plain FP64 CPU oracle for the FastLSQ hot path (test infrastructure).

Only the tests, the smoke check and the CPU-baseline leg of the benchmark may
import this package.  The product path (the HIP library and its Python binding)
never imports, links or runs anything here, and this package never imports the
product's kernels or binding.  The only shared module is the seeded input
generator, which holds no arithmetic of the method.

Layout:
  fastlsq_oracle.c  explicit loops: Eq. (2) assembly, Eq. (1)/(2) evaluation,
                    Householder-QR Tikhonov least squares, triangular solves.
  this file         ctypes loading plus the method's steps in the paper's order:
                    the linear solve of Algorithm 1 (Section 2.3), the
                    Newton-Raphson loop of Section 2.4, and the gradient of a
                    data-misfit loss through the pre-factored solve (Section 2.5
                    and the inverse heat-source application).
"""
from __future__ import annotations

import ctypes as C
import os
import subprocess
import time

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "fastlsq_oracle.c")
_LIB_PATH = os.path.join(_HERE, "liboracle.so")
_lib = None


def build(force: bool = False) -> str:
    """Compile the oracle with gcc (OpenMP)."""
    if force or not os.path.exists(_LIB_PATH) or os.path.getmtime(_LIB_PATH) < os.path.getmtime(_SRC):
        tmp = _LIB_PATH + ".tmp"
        subprocess.check_call(["gcc", "-O2", "-fopenmp", "-fPIC", "-shared", "-std=c99", "-Wall",
                               "-o", tmp, _SRC, "-lm"])
        os.replace(tmp, _LIB_PATH)
    return _LIB_PATH


def _load():
    global _lib
    if _lib is None:
        build()
        lib = C.CDLL(_LIB_PATH)
        dp = C.POINTER(C.c_double)
        ip = C.POINTER(C.c_int32)
        lib.orc_assemble.argtypes = [C.c_int, C.c_int, dp, dp, C.c_int, C.c_int64, dp, C.c_int, dp, ip,
                                     C.c_double, dp]
        lib.orc_assemble.restype = None
        lib.orc_evaluate.argtypes = [C.c_int, C.c_int, dp, dp, C.c_int, dp, C.c_int64, dp, C.c_int, ip, dp]
        lib.orc_evaluate.restype = None
        lib.orc_tikhonov.argtypes = [C.c_int64, C.c_int, dp, C.c_int, dp, C.c_double, dp, dp]
        lib.orc_tikhonov.restype = C.c_int
        lib.orc_qr_factor.argtypes = [C.c_int64, C.c_int, dp, C.c_double, dp, dp, dp]
        lib.orc_qr_factor.restype = C.c_int
        lib.orc_qr_solve.argtypes = [C.c_int64, C.c_int, dp, dp, dp, C.c_int, dp, dp]
        lib.orc_qr_solve.restype = C.c_int
        lib.orc_trisolve.argtypes = [C.c_int, dp, C.c_int, dp, C.c_int]
        lib.orc_trisolve.restype = None
        lib.orc_set_num_threads.argtypes = [C.c_int]
        lib.orc_set_num_threads.restype = None
        lib.orc_num_threads.argtypes = []
        lib.orc_num_threads.restype = C.c_int
        _lib = lib
    return _lib


def _d(a):
    return a.ctypes.data_as(C.POINTER(C.c_double))


def _i(a):
    return a.ctypes.data_as(C.POINTER(C.c_int32))


def _f64(a):
    return np.ascontiguousarray(a, dtype=np.float64)


def num_threads() -> int:
    return int(_load().orc_num_threads())


def set_num_threads(n: int) -> None:
    """OpenMP threads for the oracle's later calls (timing runs on one core or on all)."""
    _load().orc_set_num_threads(int(n))


def _terms(terms, d):
    coef = _f64([c for c, _ in terms])
    alpha = np.ascontiguousarray(np.array([list(a) for _, a in terms], dtype=np.int32).reshape(len(terms), d))
    return coef, alpha


# ---------------------------------------------------------------------------
# O1 assembly (Eq. (2), Eq. (3))
# ---------------------------------------------------------------------------

def assemble(W, b, x, terms, weight=1.0, normalize=True) -> np.ndarray:
    """A_ij = weight * (1/sqrt(N)) * sum_t c_t W_j^{alpha_t} Phi_{|alpha_t| mod 4}(W_j . x_i + b_j)."""
    W, b, x = _f64(W), _f64(b), _f64(x)
    n_feat, d = W.shape
    coef, alpha = _terms(terms, d)
    A = np.empty((x.shape[0], n_feat))
    _load().orc_assemble(d, n_feat, _d(W), _d(b), int(bool(normalize)), x.shape[0], _d(x),
                         len(terms), _d(coef), _i(alpha), float(weight), _d(A))
    return A


def assemble_system(prob, blocks=None):
    """Stack the weighted row blocks of Eq. (3): returns (A, rhs_w)."""
    blocks = prob.blocks if blocks is None else blocks
    As, rs = [], []
    for bl in blocks:
        As.append(assemble(prob.W, prob.b, bl.x, bl.terms, bl.weight, prob.normalize))
        rs.append(bl.weight * _f64(bl.rhs))
    return np.vstack(As), np.concatenate(rs)


# ---------------------------------------------------------------------------
# O3 evaluation (Eq. (1) with Eq. (2))
# ---------------------------------------------------------------------------

def evaluate(W, b, beta, xq, alphas, normalize=True) -> np.ndarray:
    """out[q, a] = D^{alpha_a} u_N(x_q); returns n_q x n_alpha."""
    W, b, beta, xq = _f64(W), _f64(b), _f64(beta), _f64(xq)
    n_feat, d = W.shape
    al = np.ascontiguousarray(np.array([list(a) for a in alphas], dtype=np.int32).reshape(len(alphas), d))
    out = np.empty((xq.shape[0], len(alphas)))
    _load().orc_evaluate(d, n_feat, _d(W), _d(b), int(bool(normalize)), _d(beta), xq.shape[0], _d(xq),
                         len(alphas), _i(al), _d(out))
    return out


def apply_operator(W, b, beta, x, terms, normalize=True) -> np.ndarray:
    """L[u_N](x) = sum_t c_t D^{alpha_t} u_N(x)."""
    vals = evaluate(W, b, beta, x, [a for _, a in terms], normalize)
    return vals @ _f64([c for c, _ in terms])


# ---------------------------------------------------------------------------
# O2 Tikhonov least squares (Section 2.3 / 2.4), Householder QR of [A; sqrt(mu) I]
# ---------------------------------------------------------------------------

def tikhonov(A, rhs, mu, return_r=False):
    """argmin ||A beta - rhs||^2 + mu ||beta||^2; rhs may be m or m x k."""
    A = _f64(A)
    m, n = A.shape
    rhs = _f64(rhs)
    vec = rhs.ndim == 1
    Y = _f64(rhs.reshape(m, -1))
    k = Y.shape[1]
    beta = np.empty((n, k))
    R = np.empty((n, n)) if return_r else None
    st = _load().orc_tikhonov(m, n, _d(A), k, _d(Y), float(mu), _d(beta),
                              _d(R) if return_r else C.cast(None, C.POINTER(C.c_double)))
    if st != 0:
        raise np.linalg.LinAlgError(f"orc_tikhonov status {st}")
    out = beta[:, 0] if vec else beta
    return (out, R) if return_r else out


class QRFactor:
    """The Householder QR of [A; sqrt(mu) I] computed once, for a matrix whose data change while
    the matrix stays (Section 2.5: the inverse application factors once).  ``solve(rhs)`` returns
    the same bits as ``tikhonov(A, rhs, mu)``; ``R`` satisfies R^T R = A^T A + mu I."""

    def __init__(self, A, mu):
        A = _f64(A)
        self.m, self.n = A.shape
        rows = self.m + self.n
        self.V = np.zeros(rows * self.n)
        self.tau = np.empty(self.n)
        self.R = np.empty((self.n, self.n))
        st = _load().orc_qr_factor(self.m, self.n, _d(A), float(mu), _d(self.V), _d(self.tau), _d(self.R))
        if st != 0:
            raise np.linalg.LinAlgError(f"orc_qr_factor status {st}")

    def solve(self, rhs):
        rhs = _f64(rhs)
        vec = rhs.ndim == 1
        Y = _f64(rhs.reshape(self.m, -1))
        k = Y.shape[1]
        beta = np.empty((self.n, k))
        st = _load().orc_qr_solve(self.m, self.n, _d(self.V), _d(self.tau), _d(self.R), k, _d(Y), _d(beta))
        if st != 0:
            raise np.linalg.LinAlgError(f"orc_qr_solve status {st}")
        return beta[:, 0] if vec else beta


def trisolve(R, Y, transpose=False):
    """Solve R x = y (or R^T x = y) with upper-triangular R; y is n or n x k."""
    R = _f64(R)
    Y = np.array(Y, dtype=np.float64, copy=True)
    vec = Y.ndim == 1
    Y2 = np.ascontiguousarray(Y.reshape(R.shape[0], -1))
    _load().orc_trisolve(R.shape[0], _d(R), Y2.shape[1], _d(Y2), int(bool(transpose)))
    return Y2[:, 0] if vec else Y2


def solve_linear(prob, timings=None):
    """Algorithm 1: assemble the augmented system of Eq. (3), then the Tikhonov solve."""
    t0 = time.perf_counter()
    A, r = assemble_system(prob)
    t1 = time.perf_counter()
    beta = tikhonov(A, r, prob.mu)
    t2 = time.perf_counter()
    if timings is not None:
        timings.update(assemble_s=t1 - t0, solve_s=t2 - t1)
    return beta


def rel_l2(a, ref):
    a, ref = np.asarray(a, dtype=np.float64), np.asarray(ref, dtype=np.float64)
    return float(np.linalg.norm(a - ref) / np.linalg.norm(ref))


# ---------------------------------------------------------------------------
# O4 Newton-Raphson (Section 2.4, Eq. (4)-(5))
# ---------------------------------------------------------------------------

def _poly(coefs, u):
    return sum(c * u ** k for k, c in enumerate(coefs))


def _dpoly(coefs, u):
    return sum(k * c * u ** (k - 1) for k, c in enumerate(coefs) if k > 0)


def newton_residual(prob, beta):
    """R_i = w * (L[u_N](x_i) + N(u_N(x_i)) - data_i) per block, stacked (Eq. (4))."""
    parts, us = [], []
    for bi, bl in enumerate(prob.blocks):
        alphas = [a for _, a in bl.terms]
        zero = tuple([0] * prob.d)
        vals = evaluate(prob.W, prob.b, beta, bl.x, alphas + [zero], prob.normalize)
        Lu = vals[:, :-1] @ _f64([c for c, _ in bl.terms])
        u = vals[:, -1]
        if bi == prob.nonlin_block:
            Lu = Lu + _poly(prob.nonlin_poly, u)
        parts.append(bl.weight * (Lu - bl.rhs))
        us.append(u)
    return np.concatenate(parts), us


def newton_jacobian(prob, us):
    """J_ij = w * (L[phi_j](x_i) + N'(u_i) phi_j(x_i) / sqrt(N)^normalize) (Section 2.4)."""
    Js = []
    zero = tuple([0] * prob.d)
    for bi, bl in enumerate(prob.blocks):
        J = assemble(prob.W, prob.b, bl.x, bl.terms, bl.weight, prob.normalize)
        if bi == prob.nonlin_block:
            H = assemble(prob.W, prob.b, bl.x, [(1.0, zero)], bl.weight, prob.normalize)
            J = J + _dpoly(prob.nonlin_poly, us[bi])[:, None] * H
        Js.append(J)
    return np.vstack(Js)


def solve_newton(prob, max_iter=15, tol_dbeta=1e-10, armijo_c=1e-4, max_halvings=10, beta0=None):
    """Gauss-Newton with Tikhonov steps, warm start and Armijo backtracking.

    Warm start: the linear solve with N dropped (Section 2.4, first refinement).
    Step: delta = argmin ||J delta + R||^2 + mu ||delta||^2 (Eq. (5)).
    Line search: halve alpha until ||R(beta + alpha delta)|| <= (1 - c alpha) ||R(beta)||,
    at most ``max_halvings`` times (then keep the smallest alpha and flag it).
    Stop when ||alpha delta||_2 < tol_dbeta.
    """
    beta = solve_linear(prob) if beta0 is None else _f64(beta0).copy()
    trace = []
    for it in range(max_iter):
        R, us = newton_residual(prob, beta)
        nR = float(np.linalg.norm(R))
        J = newton_jacobian(prob, us)
        delta = tikhonov(J, -R, prob.mu)
        alpha, halv, flagged = 1.0, 0, False
        while True:
            Rt, _ = newton_residual(prob, beta + alpha * delta)
            if np.linalg.norm(Rt) <= (1.0 - armijo_c * alpha) * nR:
                break
            if halv >= max_halvings:
                flagged = True
                break
            alpha *= 0.5
            halv += 1
        step = alpha * delta
        u_old = np.concatenate(us)
        beta = beta + step
        _, us_new = newton_residual(prob, beta)
        u_new = np.concatenate(us_new)
        trace.append(dict(it=it, res_norm=nR, alpha=alpha, halvings=halv, armijo_failed=flagged,
                          step_norm=float(np.linalg.norm(step)),
                          du_rel=float(np.linalg.norm(u_new - u_old) / max(np.linalg.norm(u_new), 1e-300))))
        if np.linalg.norm(step) < tol_dbeta:
            break
    return beta, trace


# ---------------------------------------------------------------------------
# O5 gradient of a data misfit through the pre-factored solve (Section 2.5)
# ---------------------------------------------------------------------------

def source_and_grad(x, theta):
    """s = a exp(-r^2/(2 w^2)) and ds/d(a, c_x, c_y, w) at points x (columns 0, 1 spatial)."""
    a, cx, cy, w = [float(v) for v in theta]
    dx, dy = x[:, 0] - cx, x[:, 1] - cy
    r2 = dx * dx + dy * dy
    e = np.exp(-r2 / (2.0 * w * w))
    s = a * e
    ds = np.stack([e, a * e * dx / (w * w), a * e * dy / (w * w), a * e * r2 / (w ** 3)], axis=1)
    return s, ds


class InverseOracle:
    """Forward map theta -> misfit and its gradient for the inverse heat-source workload.

    The system matrix does not depend on theta, so one QR gives R with
    R^T R = A^T A + mu I, reused for every right-hand side (Section 2.5 and the
    inverse heat-source application: factor once, two triangular solves per
    evaluation).
    """

    def __init__(self, prob, data, kappa=None):
        self.prob = prob
        self.kappa = prob.extras["kappa"] if kappa is None else kappa
        self.data = _f64(data)
        self._build()

    def _interior_terms(self, kappa):
        d = self.prob.d
        t_axis = tuple([0] * (d - 1) + [1])
        lap = []
        for k in range(d - 1):
            a = [0] * d
            a[k] = 2
            lap.append((-kappa, tuple(a)))
        return [(1.0, t_axis)] + lap

    def _build(self):
        p = self.prob
        blocks = list(p.blocks)
        blocks[0] = type(blocks[0])(blocks[0].name, blocks[0].x, self._interior_terms(self.kappa),
                                    blocks[0].weight, blocks[0].rhs)
        self.A, _ = assemble_system(p, blocks)
        d = p.d
        lap_only = []
        for k in range(d - 1):
            a = [0] * d
            a[k] = 2
            lap_only.append((-1.0, tuple(a)))
        n_int = blocks[0].n
        Ak = np.zeros_like(self.A)
        Ak[:n_int] = assemble(p.W, p.b, blocks[0].x, lap_only, blocks[0].weight, p.normalize)
        self.A_kappa = Ak
        self.qr = QRFactor(self.A, p.mu)
        self.R = self.qr.R
        self.H = assemble(p.W, p.b, p.extras["x_obs"], [(1.0, tuple([0] * d))], 1.0, p.normalize)

    def rhs(self, thetas):
        p = self.prob
        n_int = p.blocks[0].n
        m = self.A.shape[0]
        K = len(thetas)
        Rhs = np.zeros((m, K))
        dR = np.zeros((n_int, K, 4))
        for h, th in enumerate(thetas):
            s, ds = source_and_grad(p.blocks[0].x, th)
            Rhs[:n_int, h] = p.blocks[0].weight * s
            dR[:, h, :] = p.blocks[0].weight * ds
        return Rhs, dR

    def normal_solve(self, V):
        """(A^T A + mu I)^{-1} V = R^{-1} R^{-T} V."""
        return trisolve(self.R, trisolve(self.R, V, transpose=True), transpose=False)

    def loss_and_grad(self, thetas):
        """Per hypothesis: L_h = mean_k (H beta_h - d)_k^2, dL_h/dtheta_h (4), dL_h/dkappa."""
        thetas = np.atleast_2d(_f64(thetas))
        Rhs, dR = self.rhs(thetas)
        B = self.qr.solve(Rhs)                                  # N x K, the QR that gave R
        U = self.H @ B                                          # n_obs x K
        res = U - self.data[:, None]
        n_obs = U.shape[0]
        loss = np.mean(res ** 2, axis=0)
        g_u = (2.0 / n_obs) * res
        Lam = self.normal_solve(self.H.T @ g_u)                 # N x K
        AL = self.A @ Lam                                       # m x K: dL/d rhs
        n_int = dR.shape[0]
        g_theta = np.einsum("ik,ikp->kp", AL[:n_int], dR)
        r = Rhs - self.A @ B
        g_kappa = np.sum((self.A_kappa @ Lam) * r, axis=0) - np.sum(AL * (self.A_kappa @ B), axis=0)
        return loss, g_theta, g_kappa, B

    def loss(self, thetas, kappa=None):
        if kappa is not None and kappa != self.kappa:
            other = InverseOracle(self.prob, self.data, kappa)
            return other.loss(thetas)
        thetas = np.atleast_2d(_f64(thetas))
        Rhs, _ = self.rhs(thetas)
        B = self.qr.solve(Rhs)
        return np.mean((self.H @ B - self.data[:, None]) ** 2, axis=0)


# ---------------------------------------------------------------------------
# Outer optimisers: Adam (the batched source-parameter fit of the inverse heat-source
# application) and AdamW (the learnable-bandwidth appendix's hybrid training).  Adam is
# Kingma and Ba's update with bias correction; AdamW adds Loshchilov and Hutter's
# decoupled weight decay, applied to the parameters before the Adam step.
# ---------------------------------------------------------------------------

def adam_update(p, g, m, v, t, lr, b1=0.9, b2=0.999, eps=1e-8, weight_decay=0.0, clamp_col=-1, clamp_min=0.0):
    """One step at step number t >= 1 on arrays p (parameters), m, v (moments), in place:
    p <- p (1 - lr wd); m <- b1 m + (1 - b1) g; v <- b2 v + (1 - b2) g^2;
    p <- p - lr (m / (1 - b1^t)) / (sqrt(v / (1 - b2^t)) + eps); then, when clamp_col >= 0,
    p[..., clamp_col] <- max(p[..., clamp_col], clamp_min) (a projection onto w >= w_min)."""
    if weight_decay:
        p *= 1.0 - lr * weight_decay
    m *= b1
    m += (1.0 - b1) * g
    v *= b2
    v += (1.0 - b2) * g * g
    p -= lr * (m / (1.0 - b1 ** t)) / (np.sqrt(v / (1.0 - b2 ** t)) + eps)
    if clamp_col >= 0:
        col = p[..., clamp_col]
        np.maximum(col, clamp_min, out=col)
    return p


def adam_run(grad_fn, p0, steps, lr, b1=0.9, b2=0.999, eps=1e-8, weight_decay=0.0, clamp_col=-1, clamp_min=0.0):
    """``steps`` Adam(W) steps from p0 with gradients ``grad_fn(p) -> (loss, grad)``.
    Returns the parameters at the start of every step (steps x shape(p0)), the losses there,
    and the final parameters."""
    p = np.array(p0, dtype=np.float64, copy=True)
    m = np.zeros_like(p)
    v = np.zeros_like(p)
    hist_p, hist_l = [], []
    for t in range(1, steps + 1):
        loss, g = grad_fn(p)
        hist_p.append(p.copy())
        hist_l.append(np.array(loss, dtype=np.float64, copy=True))
        adam_update(p, _f64(g), m, v, t, lr, b1, b2, eps, weight_decay, clamp_col, clamp_min)
    return np.array(hist_p), np.array(hist_l), p


def adamw_sigma(grad_fn, sigma0, steps=80, lr=0.1, b1=0.9, b2=0.999, eps=1e-8, wd=0.01):
    """AdamW on the scalar bandwidth sigma (L = sigma I), ``grad_fn(sigma) -> (loss, dloss/dsigma)``;
    returns the sigma at each step's start and the loss there."""
    hist_p, hist_l, _ = adam_run(lambda p: (lambda lo, g: (lo, np.array([g])))(*grad_fn(float(p[0]))),
                                 np.array([float(sigma0)]), steps, lr, b1, b2, eps, weight_decay=wd)
    return hist_p[:, 0], hist_l


def inverse_adam(orc, theta0, steps=200, lr=1e-2, w_min=0.02):
    """The inverse heat-source fit: every hypothesis' theta = (a, c_x, c_y, w) follows Adam on its
    own misfit with the oracle's gradient, w kept >= w_min.  Returns (thetas at each step's start,
    losses there, final thetas)."""
    def gfn(th):
        loss, g, _, _ = orc.loss_and_grad(th)
        return loss, g
    return adam_run(gfn, theta0, steps, lr, clamp_col=3, clamp_min=w_min)


# ---------------------------------------------------------------------------
# Learnable bandwidth (the paper's reparameterisation appendix): W_j = L What_j with a
# lower-triangular L, outer loss ||A(L) beta*(L) - b||^2 at the Tikhonov solution
# ---------------------------------------------------------------------------

def _phi(order, z):
    """Phi_{order mod 4} of Eq. (2): sin, cos, -sin, -cos."""
    o = order % 4
    if o == 0:
        return np.sin(z)
    if o == 1:
        return np.cos(z)
    if o == 2:
        return -np.sin(z)
    return -np.cos(z)


def assemble_dW(W, b, x, terms, p, scale_j, weight=1.0, normalize=True) -> np.ndarray:
    """d A_ij / d W_jp times scale_j, written out from Eq. (2):
    d/dW_jp [W_j^alpha Phi_|alpha|(W_j . x + b_j)]
        = alpha_p W_j^(alpha - e_p) Phi_|alpha|(z) + W_j^alpha Phi_|alpha|+1(z) x_ip."""
    W, b, x = _f64(W), _f64(b), _f64(x)
    n_feat, d = W.shape
    z = x @ W.T + b[None, :]
    out = np.zeros((x.shape[0], n_feat))
    for c, a in terms:
        order = int(sum(a))
        mono = np.ones(n_feat)
        for k in range(d):
            mono = mono * W[:, k] ** a[k]
        if a[p] > 0:
            dmono = np.full(n_feat, float(a[p]))
            for k in range(d):
                dmono = dmono * W[:, k] ** (a[k] - (1 if k == p else 0))
            out += c * dmono[None, :] * _phi(order, z)
        out += c * mono[None, :] * _phi(order + 1, z) * x[:, p][:, None]
    norm = 1.0 / np.sqrt(n_feat) if normalize else 1.0
    return weight * norm * out * _f64(scale_j)[None, :]


def lower_index(d):
    """(p, q) pairs of a lower-triangular d x d matrix in packed row-major order."""
    return [(p, q) for p in range(d) for q in range(p + 1)]


def bandwidth_loss_and_grad(prob, What, L):
    """Outer loss Lo(L) = ||A beta* - b||^2 with beta* = argmin ||A beta - b||^2 + mu ||beta||^2 and
    A = A(W = What L^T), and its gradient with respect to the entries L_pq, p >= q.

    With r = b - A beta*, M = A^T A + mu I and A^T r = mu beta* (the normal equations),
    dLo/dL_pq = -2 r^T A' beta* - 2 mu beta*^T d beta*/dL_pq, and
    d beta*/dL_pq = M^{-1} (A'^T r - A^T A' beta*), so with lam = M^{-1} beta*
    dLo/dL_pq = -2 [r^T A' beta* + mu (r^T A' lam - (A lam)^T A' beta*)],  A' = dA/dL_pq.
    """
    What, L = _f64(What), _f64(L)
    d = What.shape[1]
    W = What @ L.T
    blocks = prob.blocks
    As, rs = [], []
    for bl in blocks:
        As.append(assemble(W, prob.b, bl.x, bl.terms, bl.weight, prob.normalize))
        rs.append(bl.weight * _f64(bl.rhs))
    A, rhs = np.vstack(As), np.concatenate(rs)
    beta, R = tikhonov(A, rhs, prob.mu, return_r=True)
    r = rhs - A @ beta
    loss = float(r @ r)
    lam = trisolve(R, trisolve(R, beta, transpose=True), transpose=False)
    Alam = A @ lam
    grad = []
    for p, q in lower_index(d):
        dA = np.vstack([assemble_dW(W, prob.b, bl.x, bl.terms, p, What[:, q], bl.weight, prob.normalize)
                        for bl in blocks])
        dAb = dA @ beta
        grad.append(-2.0 * (r @ dAb + prob.mu * (r @ (dA @ lam) - Alam @ dAb)))
    return loss, np.array(grad), beta


# ---------------------------------------------------------------------------
# Row-dependent coefficients (the coil operator of the applications section,
# nu Laplace u + grad nu . grad u) and nonlinearities that involve first
# derivatives (steady Burgers u u' - nu u'' of the Newton experiments, solved by
# continuation in nu as Section 2.4 describes)
# ---------------------------------------------------------------------------

def assemble_var(W, b, x, channels, weight=1.0, normalize=True) -> np.ndarray:
    """A_ij = weight * sum_t a_t(x_i) * L_t[phi_j](x_i): each channel is (terms, a) with a the
    per-row coefficient array (None = 1) and L_t the constant-coefficient operator of Eq. (2)."""
    x = _f64(x)
    A = np.zeros((x.shape[0], _f64(W).shape[0]))
    for terms, a in channels:
        At = assemble(W, b, x, terms, weight, normalize)
        A += At if a is None else _f64(a)[:, None] * At
    return A


def assemble_var_system(prob):
    As, rs = [], []
    for bl in prob.blocks:
        As.append(assemble_var(prob.W, prob.b, bl.x, bl.channels, bl.weight, prob.normalize))
        rs.append(bl.weight * _f64(bl.rhs))
    return np.vstack(As), np.concatenate(rs)


def solve_linear_var(prob):
    """The Tikhonov least-squares solve of Eq. (3) with row-dependent coefficients."""
    A, r = assemble_var_system(prob)
    return tikhonov(A, r, prob.mu)


def nonlin_grad_value(poly, adv, u, du, exp_coef=0.0):
    """N(u, grad u) = sum_k poly_k u^k + exp_coef e^u + sum_t c_t u^{m_t} d_{axis_t} u, and its
    partial derivatives: dN/du (an array) and dN/d(d_k u) per axis k (a dict)."""
    poly = tuple(poly or ())
    val = _poly(poly, u) if poly else np.zeros_like(u)
    dval_u = _dpoly(poly, u) if len(poly) > 1 else np.zeros_like(u)
    if exp_coef:
        val = val + exp_coef * np.exp(u)
        dval_u = dval_u + exp_coef * np.exp(u)
    dval_g = {}
    for c, m, ax in adv:
        g = du[ax]
        val = val + c * u ** m * g
        if m > 0:
            dval_u = dval_u + c * m * u ** (m - 1) * g
        dval_g[ax] = dval_g.get(ax, 0.0) + c * u ** m
    return val, dval_u, dval_g


def _axes(prob):
    return sorted({ax for _, _, ax in prob.nonlin_adv})


def newton_var_residual(prob, beta):
    """R_i = w (sum_t a_t(x_i) L_t[u_N](x_i) + N(u_N, grad u_N)(x_i) - data_i), stacked, with u_N
    and its first derivatives at every row of the nonlinear block; also u_N at every row."""
    d = prob.d
    zero = tuple([0] * d)
    unit = [tuple(1 if k == ax else 0 for k in range(d)) for ax in range(d)]
    parts, us = [], []
    for bi, bl in enumerate(prob.blocks):
        Lu = np.zeros(bl.x.shape[0])
        for terms, a in bl.channels:
            v = apply_operator(prob.W, prob.b, beta, bl.x, terms, prob.normalize)
            Lu = Lu + (v if a is None else _f64(a) * v)
        ev = evaluate(prob.W, prob.b, beta, bl.x, [zero] + unit, prob.normalize)
        u = ev[:, 0]
        if bi == prob.nonlin_block:
            val, _, _ = nonlin_grad_value(prob.nonlin_poly, prob.nonlin_adv, u, {k: ev[:, 1 + k] for k in range(d)},
                                       prob.nonlin_exp)
            Lu = Lu + val
        parts.append(bl.weight * (Lu - _f64(bl.rhs)))
        us.append(u)
    return np.concatenate(parts), us


def newton_var_jacobian(prob, beta):
    """J_ij = dR_i/dbeta_j: the linear rows, plus on the nonlinear block
    w (dN/du phi_j(x_i) + sum_k dN/d(d_k u) d_k phi_j(x_i)) (Section 2.4: the Jacobian keeps the
    closed form of Eq. (2))."""
    d = prob.d
    zero = tuple([0] * d)
    unit = [tuple(1 if k == ax else 0 for k in range(d)) for ax in range(d)]
    Js = []
    for bi, bl in enumerate(prob.blocks):
        J = assemble_var(prob.W, prob.b, bl.x, bl.channels, bl.weight, prob.normalize)
        if bi == prob.nonlin_block:
            ev = evaluate(prob.W, prob.b, beta, bl.x, [zero] + unit, prob.normalize)
            _, du_, dg = nonlin_grad_value(prob.nonlin_poly, prob.nonlin_adv, ev[:, 0],
                                           {k: ev[:, 1 + k] for k in range(d)}, prob.nonlin_exp)
            J = J + du_[:, None] * assemble(prob.W, prob.b, bl.x, [(1.0, zero)], bl.weight, prob.normalize)
            for ax, coef in dg.items():
                J = J + _f64(coef)[:, None] * assemble(prob.W, prob.b, bl.x, [(1.0, unit[ax])], bl.weight,
                                                       prob.normalize)
        Js.append(J)
    return np.vstack(Js)


def solve_newton_var(prob, beta0=None, max_iter=30, tol_du=1e-10, tol_dbeta=0.0, armijo_c=1e-4, max_halvings=10):
    """Newton-Raphson of Section 2.4 with its refinements: warm start from the linear part
    (nonlinearity dropped) unless beta0 is given, the Tikhonov step, Armijo backtracking on the
    residual norm, and the solution-level stop ||Delta u|| / ||u|| < tol_du at the collocation
    points (or ||alpha delta|| < tol_dbeta)."""
    beta = solve_linear_var(prob) if beta0 is None else _f64(beta0).copy()
    trace = []
    for it in range(max_iter):
        R, us = newton_var_residual(prob, beta)
        nR = float(np.linalg.norm(R))
        J = newton_var_jacobian(prob, beta)
        delta = tikhonov(J, -R, prob.mu)
        alpha, halv = 1.0, 0
        while True:
            Rt, _ = newton_var_residual(prob, beta + alpha * delta)
            if np.linalg.norm(Rt) <= (1.0 - armijo_c * alpha) * nR or halv >= max_halvings:
                break
            alpha *= 0.5
            halv += 1
        step = alpha * delta
        beta = beta + step
        u_old = np.concatenate(us)
        u_new = np.concatenate(newton_var_residual(prob, beta)[1])
        du_rel = float(np.linalg.norm(u_new - u_old) / max(np.linalg.norm(u_new), 1e-300))
        trace.append(dict(it=it, res_norm=nR, alpha=alpha, halvings=halv, step_norm=float(np.linalg.norm(step)),
                          du_rel=du_rel))
        if du_rel < tol_du or np.linalg.norm(step) < tol_dbeta:
            break
    return beta, trace


def continuation(make_problem, params, **newton_kw):
    """Homotopy (Section 2.4): solve the problems make_problem(p) for p in order, each from the
    previous solution; the first from its own linear warm start."""
    beta, traces = None, []
    for p in params:
        beta, tr = solve_newton_var(make_problem(p), beta0=beta, **newton_kw)
        traces.append(tr)
    return beta, traces
