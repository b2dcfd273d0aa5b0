"""The multi-column preconditioner application Z = X (X^T Y) (matrix-core kernels, contraction
split across workgroups) against the single-column one (vector kernels) and the oracle.

flsq_factor_solve with no refinement returns exactly (D X)(D X)^T A^T Y for the factor's inverse
factor X, so K columns at once must equal the K single-column calls up to summation order.
Feature counts straddle the kernel's chunk sizes (500, 1500, 2049 > 2048) and are not multiples
of the 16-row tiles; column counts cover 2, 17 and 64.  Each problem has mu = 0.1 (equilibrated
Gram condition number about 4e7 at 2049 features), so the unrefined solution also matches the
oracle's Householder-QR Tikhonov solution.  Bars: the rounding of the two summation orders is
bounded by n eps |D X| |X^T| |D v| (about 6e-9 of |z| here, typically far less): 1e-9 between
the two paths, 1e-7 against the oracle; an indexing mistake shows as an O(1) difference."""
import math

import numpy as np
import pytest

import oracle
from paper_2602_10541_amd import workloads as wl
from tests.gpu_util import context, rel_l2, require_gpu

pytestmark = pytest.mark.gpu


def _problem(n, seed):
    rng = np.random.default_rng(seed)
    d = 2
    W = rng.normal(0.0, 3.0, size=(n, d))
    b = rng.uniform(0, 2 * math.pi, size=n)
    n_int, n_bc = 2 * n + 37, n // 3 + 5
    xi = rng.uniform(0, 1, size=(n_int, d))
    xb = wl.sample_faces(rng, n_bc, d, range(d))
    lap = [(-1.0, (2, 0)), (-1.0, (0, 2))]
    blocks = [wl.Block("interior", xi, lap, 1.0, rng.normal(size=n_int)),
              wl.Block("boundary", xb, wl.identity_terms(d), 10.0, rng.normal(size=n_bc))]
    return wl.Problem(f"precond{n}", d, n, W, b, blocks, mu=0.1)


@pytest.mark.parametrize("n", [500, 1500, 2049])
def test_multi_column_preconditioner(n):
    torch, fl = require_gpu()
    ctx = context()
    prob = _problem(n, 4000 + n)
    dp = fl.DeviceProblem(prob)
    P = dp.n_rows
    F = fl.flsq_factorize(ctx, dp.basis, dp.rows, fl.solve_opts(prob.mu, fl.PREC_FP64, 0, 1e-12))
    assert F.info.chol_retries == 0
    A, _ = oracle.assemble_system(prob)
    qr = oracle.QRFactor(A, prob.mu)
    rng = np.random.default_rng(n)
    for K in (2, 17, 64):
        Y = rng.normal(size=(P, K))
        Yt = torch.tensor(Y, dtype=torch.float64, device="cuda")
        B = torch.empty((n, K), dtype=torch.float64, device="cuda")
        fl.flsq_factor_solve(ctx, F, Yt, B)
        got = B.cpu().numpy()
        ref = qr.solve(Y)
        for s in sorted({0, K // 2, K - 1}):
            b1 = torch.empty(n, dtype=torch.float64, device="cuda")
            fl.flsq_factor_solve(ctx, F, Yt[:, s].contiguous(), b1)
            assert rel_l2(got[:, s], b1.cpu().numpy()) <= 1e-9, (n, K, s)
        errs = [rel_l2(got[:, s], ref[:, s]) for s in range(K)]
        assert max(errs) <= 1e-7, (n, K, max(errs))
    F.free()


@pytest.mark.parametrize("n", [500, 2049])
def test_stored_matrix_products(n):
    """A factor that keeps A and A^T: its 17..64-column products (matrix-core GEMM over the stored
    rows, split contraction) against the oracle's assembled matrix, entry by entry within 1e-12
    of |A| |V| (the FP64 rounding scale), and its refined multi-column solves against the
    matrix-free factor's and the oracle's."""
    torch, fl = require_gpu()
    ctx = context()
    prob = _problem(n, 7000 + n)
    dp = fl.DeviceProblem(prob)
    P = dp.n_rows
    A, _ = oracle.assemble_system(prob)
    Fd = fl.flsq_factorize(ctx, dp.basis, dp.rows, fl.solve_opts(prob.mu, fl.PREC_FP64, 10, 1e-13, store_matrix=True))
    Fm = fl.flsq_factorize(ctx, dp.basis, dp.rows, fl.solve_opts(prob.mu, fl.PREC_FP64, 10, 1e-13))
    rng = np.random.default_rng(n + 1)
    for K in (17, 40, 64):
        V = rng.normal(size=(n, K))
        Y = rng.normal(size=(P, K))
        Vt = torch.tensor(V, dtype=torch.float64, device="cuda")
        Yt = torch.tensor(Y, dtype=torch.float64, device="cuda")
        AV = torch.empty((P, K), dtype=torch.float64, device="cuda")
        AtY = torch.empty((n, K), dtype=torch.float64, device="cuda")
        fl.flsq_apply_A(ctx, Fd, Vt, AV)
        fl.flsq_apply_At(ctx, Fd, Yt, AtY)
        assert np.abs(AV.cpu().numpy() - A @ V).max() <= 1e-12 * (np.abs(A) @ np.abs(V)).max(), (n, K)
        assert np.abs(AtY.cpu().numpy() - A.T @ Y).max() <= 1e-12 * (np.abs(A).T @ np.abs(Y)).max(), (n, K)
        Bd = torch.empty((n, K), dtype=torch.float64, device="cuda")
        Bm = torch.empty((n, K), dtype=torch.float64, device="cuda")
        fl.flsq_factor_solve(ctx, Fd, Yt, Bd)
        fl.flsq_factor_solve(ctx, Fm, Yt, Bm)
        ref = oracle.tikhonov(A, Y[:, :3], prob.mu)
        assert rel_l2(Bd.cpu().numpy(), Bm.cpu().numpy()) <= 1e-10, (n, K)
        for s in range(3):
            assert rel_l2(Bd.cpu().numpy()[:, s], ref[:, s]) <= 1e-10, (n, K, s)
    Fd.free()
    Fm.free()
