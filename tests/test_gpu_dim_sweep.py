"""GPU parity sweep over every dimension the library instantiates (d = 1 .. 8), fixed seeds.

Each case draws features, a random interior operator of up to three terms with |alpha| <= 4
(odd and even orders mixed, so both the folded amplitude/phase form and the sine-only form
run), an identity boundary block, and feature and row counts that are not multiples of any
tile, run or chunk size.  Against the oracle on the same inputs: the assembled matrix (FP64
and FP32), the Gram in every precision, the matrix-free products A V and A^T Y for one, a
few and many columns (the VALU and the matrix-core pass kernels), a Tikhonov solve, and the
evaluation of mixed sine/cosine-type derivatives in FP64 and FP32.
"""
import math

import numpy as np
import pytest

import oracle
from paper_2602_10541_amd import workloads as wl
from tests.gpu_util import amplitude_bound, context, rel_l2, require_gpu

pytestmark = pytest.mark.gpu
DIMS = list(range(1, 9))


def _random_alpha(rng, d, max_order=4):
    order = int(rng.integers(0, max_order + 1))
    a = [0] * d
    for _ in range(order):
        a[int(rng.integers(0, d))] += 1
    return tuple(a)


def _problem(d, mu=1e-6):
    rng = np.random.default_rng(1000 + d)
    n = 129 + 37 * d
    n_int, n_bc = 301 + 17 * d, 67 + 5 * d
    sigma = 2.0 / math.sqrt(d)
    W = rng.normal(0.0, sigma, size=(n, d))
    b = rng.uniform(0, 2 * math.pi, size=n)
    terms = [(float(rng.uniform(-2, 2)), _random_alpha(rng, d)) for _ in range(1 + d % 3)]
    terms.append((1.0, tuple([1 if k == d - 1 else 0 for k in range(d)])))   # at least one odd order
    xi = rng.uniform(0, 1, size=(n_int, d))
    xb = wl.sample_faces(rng, n_bc, d, range(d))
    blocks = [wl.Block("interior", xi, terms, 1.0, rng.normal(size=n_int)),
              wl.Block("boundary", xb, wl.identity_terms(d), 10.0, rng.normal(size=n_bc))]
    return wl.Problem(f"sweep{d}", d, n, W, b, blocks, mu=mu)


@pytest.mark.parametrize("d", DIMS)
def test_dimension_sweep(d):
    torch, fl = require_gpu()
    ctx = context()
    prob = _problem(d)
    dp = fl.DeviceProblem(prob)
    P, N = dp.n_rows, prob.n_feat
    A_ref, r_ref = oracle.assemble_system(prob)

    # assembly, FP64 and FP32, scaled per entry by the block's amplitude bound
    for fp32, bar in ((False, 1e-12), (True, 1e-5)):
        A = torch.empty((P, N), dtype=torch.float32 if fp32 else torch.float64, device="cuda")
        fl.flsq_assemble(ctx, dp.basis, dp.rows, A, None, fp32=fp32)
        A = A.double().cpu().numpy()
        r0 = 0
        for bl in prob.blocks:
            s = amplitude_bound(prob.W, bl.terms, bl.weight)
            e = np.abs(A[r0:r0 + bl.n] - A_ref[r0:r0 + bl.n]) / s[None, :]
            assert e.max() <= bar, (d, bl.name, fp32, e.max())
            r0 += bl.n

    # Gram in every precision
    G_ref = A_ref.T @ A_ref
    for prec, bar in ((0, 1e-13), (1, 2e-6), (2, 1e-4), (3, 5e-13)):
        G = torch.empty((N, N), dtype=torch.float64, device="cuda")
        c = torch.empty(N, dtype=torch.float64, device="cuda")
        fl.flsq_gram(ctx, dp.basis, dp.rows, prec, G, c)
        err = np.linalg.norm(G.cpu().numpy() - G_ref) / np.linalg.norm(G_ref)
        assert err <= bar, (d, prec, err)
        assert rel_l2(c.cpu().numpy(), A_ref.T @ r_ref) <= 1e-13

    # matrix-free products for 1, 3, 17 and 40 columns
    F = fl.flsq_factorize(ctx, dp.basis, dp.rows, fl.solve_opts(prob.mu, 0, 30, 1e-12))
    rng = np.random.default_rng(d)
    for K in (1, 3, 17, 40):
        V = rng.normal(size=(N, K))
        Y = rng.normal(size=(P, K))
        Vt = torch.tensor(V[:, 0] if K == 1 else V, dtype=torch.float64, device="cuda")
        Yt = torch.tensor(Y[:, 0] if K == 1 else Y, dtype=torch.float64, device="cuda")
        AV = torch.empty((P,) if K == 1 else (P, K), dtype=torch.float64, device="cuda")
        AtY = torch.empty((N,) if K == 1 else (N, K), dtype=torch.float64, device="cuda")
        fl.flsq_apply_A(ctx, F, Vt, AV)
        fl.flsq_apply_At(ctx, F, Yt, AtY)
        ref_av, ref_aty = A_ref @ V, A_ref.T @ Y
        got_av = AV.cpu().numpy().reshape(P, K)
        got_aty = AtY.cpu().numpy().reshape(N, K)
        assert np.abs(got_av - ref_av).max() <= 1e-12 * (np.abs(A_ref) @ np.abs(V)).max(), (d, K)
        assert np.abs(got_aty - ref_aty).max() <= 1e-12 * (np.abs(A_ref).T @ np.abs(Y)).max(), (d, K)
    F.free()

    # Tikhonov solve (mu = 1e-6): fitted values against the oracle's QR solution
    beta = torch.empty(N, dtype=torch.float64, device="cuda")
    st, info = fl.flsq_solve_linear(ctx, dp.basis, dp.rows, fl.solve_opts(prob.mu, 3, 60, 1e-13), beta)
    assert st == fl.FLSQ_OK, (d, info.as_dict())
    bref = oracle.tikhonov(A_ref, r_ref, prob.mu)
    assert rel_l2(A_ref @ beta.cpu().numpy(), A_ref @ bref) <= 1e-9, (d, info.as_dict())

    # evaluation of several derivatives of mixed type, FP64 and FP32
    alphas = [tuple([0] * d)] + [_random_alpha(rng, d, 3) for _ in range(min(7, 1 + d))]
    xq = rng.uniform(0, 1, size=(777, d))
    bq = rng.normal(size=N)
    bt = torch.tensor(bq, dtype=torch.float64, device="cuda")
    for fp32, bar in ((False, 1e-12), (True, 1e-5)):
        dt = torch.float32 if fp32 else torch.float64
        xt = torch.tensor(xq, dtype=dt, device="cuda")
        out = torch.empty((xq.shape[0], len(alphas)), dtype=dt, device="cuda")
        fl.flsq_evaluate(ctx, dp.basis, bt, xt, alphas, out)
        xr = xq.astype(np.float32).astype(np.float64) if fp32 else xq
        ref = oracle.evaluate(prob.W, prob.b, bq, xr, alphas)
        got = out.double().cpu().numpy()
        for a, al in enumerate(alphas):
            mono = np.prod(np.abs(prob.W) ** np.array(al)[None, :], axis=1)
            scale = np.sum(np.abs(bq) * mono) / math.sqrt(N)
            e = np.abs(got[:, a] - ref[:, a]).max() / scale
            assert e <= bar, (d, fp32, al, e)
