"""GPU parity of the linear path (assembly, Gram, Tikhonov solve, evaluation) against the CPU oracle.

Every test calls the HIP library through its C ABI (ctypes binding) and compares
with the oracle on the same seeded inputs.  Bars: scaled entry error <= 1e-12
(FP64) / 1e-5 (FP32); u at the 5000 test points within 1e-7 relative L2 of the
oracle's Householder-QR solution for the FP64 path.
"""
import math
import os

import numpy as np
import pytest

import oracle
from paper_2602_10541_amd import workloads as wl
from tests.gpu_util import pde_residual, amplitude_bound, context, rel_l2, require_gpu

pytestmark = pytest.mark.gpu
GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden")


def _small_problems():
    # several 128-feature tiles with a ragged tail, blocks not multiples of 32 / 64 rows
    return [
        wl.poisson(2, 300, 3.0, 1000, 237, seed=1, name="p2", n_test=500),
        wl.poisson(6, 333, 2.0, 777, 301, seed=2, name="p6", n_test=500),
        wl.heat(n_feat=257, n_int=900, n_ic=133, n_bc=190, n_query=0, seed=3, n_test=500),
        wl.inverse_heat(n_feat=130, n_int=500, n_ic=70, n_bc=65, n_obs=50, n_hyp=4, seed=4),
    ]


def _dev(prob):
    _, fl = require_gpu()
    return fl.DeviceProblem(prob)


@pytest.mark.parametrize("fp32", [False, True])
def test_assembly_matches_oracle(fp32):
    torch, fl = require_gpu()
    ctx = context()
    for prob in _small_problems():
        dp = _dev(prob)
        P, N = dp.n_rows, prob.n_feat
        A = torch.empty((P, N), dtype=torch.float32 if fp32 else torch.float64, device="cuda")
        rhs = torch.empty(P, dtype=torch.float64, device="cuda")
        fl.flsq_assemble(ctx, dp.basis, dp.rows, A, rhs, fp32=fp32)
        A = A.double().cpu().numpy()
        r0 = 0
        for bl in prob.blocks:
            ref = oracle.assemble(prob.W, prob.b, bl.x, bl.terms, bl.weight, prob.normalize)
            s = amplitude_bound(prob.W, bl.terms, bl.weight, prob.normalize)
            e = np.abs(A[r0:r0 + bl.n] - ref) / np.maximum(s, 1e-300)[None, :]
            bar = 1e-5 if fp32 else 1e-12
            assert e.max() <= bar, (prob.name, bl.name, fp32, e.max())
            r0 += bl.n
        ref_rhs = np.concatenate([bl.weight * bl.rhs for bl in prob.blocks])
        np.testing.assert_array_equal(rhs.cpu().numpy(), ref_rhs)


def test_sin_accuracy_wide_phase():
    """sin(w x + b) for |z| up to ~400 against numpy's double sin (identity operator, no normalisation)."""
    torch, fl = require_gpu()
    ctx = context()
    rng = np.random.default_rng(0)
    W = rng.uniform(-200, 200, size=(512, 1))
    b = rng.uniform(0, 2 * math.pi, size=512)
    x = rng.uniform(0, 1, size=(96, 1))
    Wt = torch.tensor(W, dtype=torch.float64, device="cuda")
    bt = torch.tensor(b, dtype=torch.float64, device="cuda")
    xt = torch.tensor(x, dtype=torch.float64, device="cuda")
    basis = fl.make_basis(Wt, bt, normalize=False)
    rows = fl.make_rows([(xt, [(1.0, (0,))], 1.0, None)], 1)
    for fp32, tol in ((False, 2e-15), (True, 1e-6)):
        A = torch.empty((96, 512), dtype=torch.float32 if fp32 else torch.float64, device="cuda")
        fl.flsq_assemble(ctx, basis, rows, A, None, fp32=fp32)
        z = x @ W.T + b
        if fp32:  # the float32 phase the kernel forms: round(w x) + b, both in float32
            z = ((x.astype(np.float32) @ W.T.astype(np.float32)) + b.astype(np.float32)[None, :]).astype(np.float64)
        err = np.abs(A.double().cpu().numpy() - np.sin(z))
        assert err.max() <= tol, (fp32, err.max())


@pytest.mark.parametrize("prec", [0, 1, 2, 3])
def test_gram_matches_oracle(prec):
    torch, fl = require_gpu()
    ctx = context()
    for prob in _small_problems():
        dp = _dev(prob)
        N = prob.n_feat
        G = torch.empty((N, N), dtype=torch.float64, device="cuda")
        c = torch.empty(N, dtype=torch.float64, device="cuda")
        fl.flsq_gram(ctx, dp.basis, dp.rows, prec, G, c)
        A, r = oracle.assemble_system(prob)
        Gref = A.T @ A
        Gg = G.cpu().numpy()
        err = np.linalg.norm(Gg - Gref) / np.linalg.norm(Gref)
        # INT8_CRT rounds each entry to >= 41 bits of its feature's amplitude bound (|delta| <=
        # 2^-42 c_j); the Gram error is then a few 1e-13 of ||G||_F at most.
        # BF16x3 keeps hi.hi + hi.lo + lo.hi of a 2 x 8-bit split: about 2^-16 per product.
        bar = {0: 1e-13, 1: 2e-6, 2: 1e-4, 3: 5e-13}[prec]
        assert err <= bar, (prob.name, prec, err)
        np.testing.assert_allclose(Gg, Gg.T, rtol=0, atol=0)
        cref = A.T @ r
        assert rel_l2(c.cpu().numpy(), cref) <= 1e-13


@pytest.mark.parametrize("n_int,n_bc", [(40, 10), (150, 40), (300, 83)])
def test_int8_gram_few_row_blocks(n_int, n_bc):
    """INT8_CRT Gram with 2, 4 and 6 K blocks of 64 rows (rows padded to a multiple of 128):
    fewer blocks than the load ring has slots, so the pipeline's refills past the last block
    are all that fill some slots; two 256-feature tiles with a ragged tail."""
    torch, fl = require_gpu()
    ctx = context()
    prob = wl.poisson(2, 300, 3.0, n_int, n_bc, seed=9, name="p2few", n_test=10)
    dp = _dev(prob)
    N = prob.n_feat
    G = torch.empty((N, N), dtype=torch.float64, device="cuda")
    c = torch.empty(N, dtype=torch.float64, device="cuda")
    fl.flsq_gram(ctx, dp.basis, dp.rows, 3, G, c)
    A, r = oracle.assemble_system(prob)
    Gref = A.T @ A
    Gg = G.cpu().numpy()
    assert np.linalg.norm(Gg - Gref) / np.linalg.norm(Gref) <= 5e-13
    np.testing.assert_allclose(Gg, Gg.T, rtol=0, atol=0)
    assert rel_l2(c.cpu().numpy(), A.T @ r) <= 1e-13


def _solve(dp, prob, prec=0, max_refine=10, tol=1e-12, keep=None):
    torch, fl = require_gpu()
    ctx = context()
    beta = torch.empty(prob.n_feat, dtype=torch.float64, device="cuda")
    st, info = fl.flsq_solve_linear(ctx, dp.basis, dp.rows, fl.solve_opts(prob.mu, prec, max_refine, tol), beta)
    if keep is not None:
        keep.append(beta)
    return st, info, beta.cpu().numpy()


def _check_pde_residual(dp, prob, beta_dev, cfg, tol):
    """The PDE residual on the test set of the GPU solution against the oracle solution's."""
    torch, fl = require_gpu()
    g = np.load(os.path.join(GOLDEN, "pde_residuals.npz"))
    r = pde_residual(fl, context(), dp, prob, beta_dev)
    scale = np.linalg.norm(prob.extras["residual_scale_test"])
    dev = np.linalg.norm(r - g[f"{cfg}_residual"]) / scale
    assert dev <= tol, (cfg, dev, np.linalg.norm(r) / scale, float(g[f"{cfg}_rel"]))
    return dev


@pytest.mark.parametrize("prec", [0, 3])
@pytest.mark.parametrize("idx", [0, 1, 2])
def test_solve_linear_small_matches_oracle(idx, prec):
    prob = _small_problems()[idx]
    dp = _dev(prob)
    st, info, beta = _solve(dp, prob, prec=prec, max_refine=30)
    torch, fl = require_gpu()
    assert st == fl.FLSQ_OK, (prob.name, info.as_dict())
    ref = oracle.solve_linear(prob)
    zero = [tuple([0] * prob.d)]
    u = oracle.evaluate(prob.W, prob.b, beta, prob.x_test, zero)[:, 0]
    uref = oracle.evaluate(prob.W, prob.b, ref, prob.x_test, zero)[:, 0]
    assert rel_l2(u, uref) <= 1e-7, (prob.name, rel_l2(u, uref), info.as_dict())
    # first-order optimality of the Tikhonov problem, checked with the oracle's assembly
    A, r = oracle.assemble_system(prob)
    g = A.T @ (r - A @ beta) - prob.mu * beta
    assert np.linalg.norm(g) <= 1e-8 * np.linalg.norm(A.T @ r)


@pytest.mark.parametrize("prec", [0, 3])
def test_solve_linear_poisson2d_full(prec):
    """2D Poisson, N = 500, 2000 + 400 rows: FP64 end to end, and the int8-CRT Gram."""
    prob = wl.config("poisson2d")
    dp = _dev(prob)
    keep = []
    st, info, beta = _solve(dp, prob, prec=prec, max_refine=30, keep=keep)
    torch, fl = require_gpu()
    assert st == fl.FLSQ_OK, info.as_dict()
    gold = np.load(os.path.join(GOLDEN, "poisson2d.npz"))
    u = oracle.evaluate(prob.W, prob.b, beta, prob.x_test, [(0, 0)])[:, 0]
    assert rel_l2(u, gold["u_test"]) <= 1e-7, (rel_l2(u, gold["u_test"]), info.as_dict())
    assert rel_l2(u, prob.u_test) <= 1e-6
    _check_pde_residual(dp, prob, keep[0], "poisson2d", 1e-6)


@pytest.mark.parametrize("prec", [0, 3])
def test_pivot_boost_factors_without_restart(prec):
    """The opt-in modified Cholesky on the 2D Poisson Gram (whose equilibrated Gram has pivots
    below 1e-13): no restart, the raised pivots counted, the automatic second pass taken, and the
    oracle's solution reached; an out-of-range boost is refused."""
    torch, fl = require_gpu()
    prob = wl.config("poisson2d")
    dp = _dev(prob)
    ctx = context()
    beta = torch.empty(prob.n_feat, dtype=torch.float64, device="cuda")
    st, info = fl.flsq_solve_linear(ctx, dp.basis, dp.rows, fl.solve_opts(prob.mu, prec, 30, 1e-12, pivot_boost=1e-13),
                                    beta)
    assert st == fl.FLSQ_OK, info.as_dict()
    assert info.chol_retries == 0 and info.boosted_pivots > 0 and info.second_pass == 1, info.as_dict()
    gold = np.load(os.path.join(GOLDEN, "poisson2d.npz"))
    u = oracle.evaluate(prob.W, prob.b, beta.cpu().numpy(), prob.x_test, [(0, 0)])[:, 0]
    assert rel_l2(u, gold["u_test"]) <= 1e-7, (rel_l2(u, gold["u_test"]), info.as_dict())
    with pytest.raises(fl.FlsqError) as ei:
        fl.flsq_solve_linear(ctx, dp.basis, dp.rows, fl.solve_opts(prob.mu, prec, 30, 1e-12, pivot_boost=1.5), beta)
    assert ei.value.status == fl.FLSQ_EINVAL


@pytest.mark.parametrize("prec", [0, 3])
def test_solve_linear_poisson6d_full(prec):
    """6D Poisson at full size (N = 4096, 32768 + 8192 rows): FP64 and int8-CRT Gram paths vs the
    oracle's stored solution."""
    path = os.path.join(GOLDEN, "poisson6d.npz")
    if not os.path.exists(path):
        pytest.skip("golden values not generated")
    prob = wl.config("poisson6d")
    dp = _dev(prob)
    keep = []
    st, info, beta = _solve(dp, prob, prec=prec, max_refine=30, keep=keep)
    torch, fl = require_gpu()
    assert st == fl.FLSQ_OK, info.as_dict()
    _check_pde_residual(dp, prob, keep[0], "poisson6d", 1e-6)
    gold = np.load(path)
    u = oracle.evaluate(prob.W, prob.b, beta, prob.x_test, [tuple([0] * 6)])[:, 0]
    assert rel_l2(u, gold["u_test"]) <= 1e-7, (rel_l2(u, gold["u_test"]), info.as_dict())
    A, r = oracle.assemble_system(prob)
    res = A @ beta - r
    obj = res @ res + prob.mu * beta @ beta
    assert obj <= float(gold["objective"]) * (1 + 1e-9)


@pytest.mark.parametrize("prec", [1, 2])
def test_fp32_preconditioned_path_well_conditioned(prec):
    """FP32 and BF16x3 Grams as preconditioners reach the FP64 answer on a well-conditioned 6D case."""
    prob = wl.poisson(6, 512, 2.0, 4000, 1000, seed=5, name="p6w", n_test=500)
    dp = _dev(prob)
    st, info, beta = _solve(dp, prob, prec=prec, max_refine=80, tol=1e-13)
    ref = oracle.solve_linear(prob)
    u = oracle.evaluate(prob.W, prob.b, beta, prob.x_test, [tuple([0] * 6)])[:, 0]
    uref = oracle.evaluate(prob.W, prob.b, ref, prob.x_test, [tuple([0] * 6)])[:, 0]
    assert rel_l2(u, uref) <= 1e-7, (rel_l2(u, uref), info.as_dict())


@pytest.mark.parametrize("prec", [1, 2])
def test_fp32_paths_reach_the_bar_on_poisson2d(prec):
    """The FP32-MFMA (and BF16x3) Gram as the preconditioner of FP64 CGLS on the 2D Poisson
    config: the shifted factor leaves a slowly converging refinement, so the step-size stop
    must be tighter than the 1e-10 used with the exact Grams.  At a 1e-11 stop FP32 takes about
    420 steps and BF16x3 about 430, and both end within 1e-7 of the oracle's solution (about
    7e-9 and 1.4e-8).  At a 1e-10 stop the slow rate stops them after 90 to 230 steps, between
    7e-8 and 1.4e-7 depending on the order of the terms in the factor's sums.  On the 6D
    Poisson and 3D + t heat configs the same paths stall above 1e-3 after 300 steps."""
    torch, fl = require_gpu()
    prob = wl.config("poisson2d")
    dp = _dev(prob)
    st, info, beta = _solve(dp, prob, prec=prec, max_refine=600, tol=1e-11)
    assert st == fl.FLSQ_OK, info.as_dict()
    gold = np.load(os.path.join(GOLDEN, "poisson2d.npz"))
    u = oracle.evaluate(prob.W, prob.b, beta, prob.x_test, [(0, 0)])[:, 0]
    assert rel_l2(u, gold["u_test"]) <= 1e-7, (rel_l2(u, gold["u_test"]), info.as_dict())


@pytest.mark.parametrize("fp32", [False, True])
def test_evaluate_matches_oracle(fp32):
    torch, fl = require_gpu()
    ctx = context()
    rng = np.random.default_rng(9)
    for d, N, Q in ((2, 300, 1000), (4, 257, 777), (6, 129, 513)):
        W = rng.normal(0, 3, size=(N, d))
        b = rng.uniform(0, 2 * math.pi, N)
        beta = rng.normal(size=N)
        xq = rng.uniform(0, 1, size=(Q, d))
        alphas = [tuple([0] * d)] + [tuple(1 if i == k else 0 for i in range(d)) for k in range(d)]
        alphas.append(tuple([2] + [0] * (d - 1)))
        alphas = alphas[:8]
        ref = oracle.evaluate(W, b, beta, xq, alphas)
        Wt = torch.tensor(W, dtype=torch.float64, device="cuda")
        bt = torch.tensor(b, dtype=torch.float64, device="cuda")
        bet = torch.tensor(beta, dtype=torch.float64, device="cuda")
        dt = torch.float32 if fp32 else torch.float64
        xt = torch.tensor(xq, dtype=dt, device="cuda")
        out = torch.empty((Q, len(alphas)), dtype=dt, device="cuda")
        fl.flsq_evaluate(ctx, fl.make_basis(Wt, bt), bet, xt, alphas, out)
        got = out.double().cpu().numpy()
        # scale of output a: norm * sum_j |beta_j| |W_j^alpha|
        for a, al in enumerate(alphas):
            mono = np.prod(np.abs(W) ** np.array(al)[None, :], axis=1)
            scale = np.sum(np.abs(beta) * mono) / math.sqrt(N)
            if fp32:
                xr = xq.astype(np.float32).astype(np.float64)
                ref_a = oracle.evaluate(W, b, beta, xr, [al])[:, 0]
                bar = 2e-5
            else:
                ref_a = ref[:, a]
                bar = 1e-13
            e = np.abs(got[:, a] - ref_a).max() / scale
            assert e <= bar, (d, al, fp32, e)


# ----------------------------------------------------------------------------- failure handling

def test_rejects_multi_index_beyond_d():
    torch, fl = require_gpu()
    ctx = context()
    prob = wl.poisson(2, 64, 2.0, 100, 20, seed=1, n_test=10)
    dp = _dev(prob)
    bad = fl.make_rows([(dp.xs[0], [(1.0, (0, 0, 1))], 1.0, dp.rhs[0])], 2)
    beta = torch.empty(64, dtype=torch.float64, device="cuda")
    with pytest.raises(fl.FlsqError) as ei:
        fl.flsq_solve_linear(ctx, dp.basis, bad, fl.solve_opts(1e-10), beta)
    assert ei.value.status == fl.FLSQ_EINVAL


def test_rejects_nan_points():
    torch, fl = require_gpu()
    ctx = context()
    prob = wl.poisson(2, 64, 2.0, 100, 20, seed=1, n_test=10)
    prob.blocks[0].x[5, 1] = float("nan")
    dp = _dev(prob)
    beta = torch.empty(64, dtype=torch.float64, device="cuda")
    with pytest.raises(fl.FlsqError) as ei:
        fl.flsq_solve_linear(ctx, dp.basis, dp.rows, fl.solve_opts(1e-10), beta)
    assert ei.value.status == fl.FLSQ_ENONFINITE


def test_duplicated_features_without_tikhonov():
    """mu = 0 with two identical features: the Gram is singular; the solve shifts or reports ENOTSPD."""
    torch, fl = require_gpu()
    ctx = context()
    prob = wl.poisson(2, 64, 2.0, 300, 60, seed=1, n_test=10)
    prob.W[1] = prob.W[0]
    prob.b[1] = prob.b[0]
    prob.mu = 0.0
    dp = _dev(prob)
    beta = torch.empty(64, dtype=torch.float64, device="cuda")
    st, info = fl.flsq_solve_linear(ctx, dp.basis, dp.rows, fl.solve_opts(0.0, 0, 5, 1e-12), beta, check=False)
    assert st in (fl.FLSQ_OK, fl.FLSQ_ENOTSPD, fl.FLSQ_ENOCONV)
    if st != fl.FLSQ_ENOTSPD:
        assert (info.chol_retries >= 1 or info.shift_recalled == 1) and info.shift > 0
        assert np.all(np.isfinite(beta.cpu().numpy()))


def test_max_refine_limit_reports_noconv():
    torch, fl = require_gpu()
    ctx = context()
    prob = wl.poisson(6, 256, 2.0, 2000, 500, seed=1, n_test=10)
    dp = _dev(prob)
    beta = torch.empty(256, dtype=torch.float64, device="cuda")
    st, info = fl.flsq_solve_linear(ctx, dp.basis, dp.rows, fl.solve_opts(1e-10, 1, 1, 1e-30), beta, check=False)
    assert st == fl.FLSQ_ENOCONV and info.refine_iters == 1


def test_int8_crt_rejects_too_many_rows():
    """The int8 Gram needs exact int32 sums of 127^2-bounded products: at most 133 000 rows."""
    torch, fl = require_gpu()
    prob = wl.poisson(2, 64, 3.0, 140000, 1000, seed=9, name="big", n_test=10)
    dp = _dev(prob)
    ctx = context()
    beta = torch.empty(prob.n_feat, dtype=torch.float64, device="cuda")
    st, info = fl.flsq_solve_linear(ctx, dp.basis, dp.rows, fl.solve_opts(prob.mu, 3), beta, check=False)
    assert st == fl.FLSQ_EINVAL and "133000" in ctx.last_error()
