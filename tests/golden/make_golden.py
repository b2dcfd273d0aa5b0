"""Write the oracle's full-size reference values used by the GPU parity tests.

Calls only the CPU oracle (oracle/) and the seeded workload generator; nothing
from the HIP path.  Usage: python tests/golden/make_golden.py [name ...]
Outputs tests/golden/<name>.npz (float64 arrays, no pickles).
"""
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

import oracle  # noqa: E402
from paper_2602_10541_amd import workloads as wl  # noqa: E402

OUT = os.path.dirname(os.path.abspath(__file__))


def linear(name):
    prob = wl.config(name)
    t = {}
    beta = oracle.solve_linear(prob, t)
    u = oracle.evaluate(prob.W, prob.b, beta, prob.x_test, [tuple([0] * prob.d)])[:, 0]
    A, r = oracle.assemble_system(prob)
    res = A @ beta - r
    obj = float(res @ res + prob.mu * beta @ beta)
    np.savez(os.path.join(OUT, f"{name}.npz"), beta=beta, u_test=u, objective=np.array(obj),
             err_exact=np.array(oracle.rel_l2(u, prob.u_test)), assemble_s=np.array(t["assemble_s"]),
             solve_s=np.array(t["solve_s"]), threads=np.array(oracle.num_threads()))
    print(name, "objective", obj, "rel err vs exact", oracle.rel_l2(u, prob.u_test), t, flush=True)


def newton(name):
    prob = wl.config(name)
    beta, trace = oracle.solve_newton(prob, max_iter=15)
    u = oracle.evaluate(prob.W, prob.b, beta, prob.x_test, [tuple([0] * prob.d)])[:, 0]
    np.savez(os.path.join(OUT, f"{name}.npz"), beta=beta, u_test=u,
             res_norm=np.array([t["res_norm"] for t in trace]), alpha=np.array([t["alpha"] for t in trace]),
             step_norm=np.array([t["step_norm"] for t in trace]), err_exact=np.array(oracle.rel_l2(u, prob.u_test)))
    print(name, "steps", len(trace), "res", [t["res_norm"] for t in trace], "err", oracle.rel_l2(u, prob.u_test),
          flush=True)


def inverse(name):
    """Observations from the oracle's forward solve at the true source, plus 1 % relative noise."""
    prob = wl.config(name)
    n_obs = prob.extras["x_obs"].shape[0]
    orc0 = oracle.InverseOracle(prob, np.zeros(n_obs))
    rhs_true = orc0.rhs([wl.THETA_TRUE])[0][:, 0]
    u_true = orc0.H @ oracle.tikhonov(orc0.A, rhs_true, prob.mu)
    data = wl.add_noise(u_true, prob.extras["noise"])
    orc = oracle.InverseOracle(prob, data)
    loss, g, gk, _ = orc.loss_and_grad(prob.extras["theta0"])
    np.savez(os.path.join(OUT, f"{name}.npz"), data=data, u_true=u_true, loss0=loss, grad_theta0=g, grad_kappa0=gk)
    print(name, "loss0[:4]", loss[:4], flush=True)


ADAM_CHECKPOINTS = (0, 1, 2, 5, 10, 20, 50, 100, 150, 199)


def inverse_adam(name):
    """The workload's 200 batched Adam steps (lr 1e-2, w >= 0.02) for all 64 hypotheses on the
    oracle's gradients, from the stored noisy observations: theta at a few step starts, every
    loss, the final theta."""
    prob = wl.config("inverse3d")
    gold = np.load(os.path.join(OUT, "inverse3d.npz"))
    t0 = time.time()
    orc = oracle.InverseOracle(prob, gold["data"])
    t_fac = time.time() - t0
    t0 = time.time()
    hist, losses, final = oracle.inverse_adam(orc, prob.extras["theta0"], steps=200, lr=1e-2, w_min=0.02)
    t_run = time.time() - t0
    ck = np.array(ADAM_CHECKPOINTS)
    np.savez(os.path.join(OUT, f"{name}.npz"), checkpoints=ck, theta_at=hist[ck], losses=losses, theta_final=final,
             factor_s=np.array(t_fac), run_s=np.array(t_run), threads=np.array(oracle.num_threads()))
    best = int(np.argmin(losses[-1]))
    print(name, "best hypothesis", best, final[best], "loss", losses[-1][best], "factor", t_fac, "s, 200 steps",
          t_run, "s", flush=True)


def reaction2d_timing(name):
    """One-core oracle times of the reaction-diffusion workload (the paper's single-core setting): the
    linear warm start (assembly + Householder QR) and the first Gauss-Newton step."""
    prob = wl.config("reaction2d")
    oracle.set_num_threads(1)
    t = {}
    t0 = time.time()
    beta = oracle.solve_linear(prob, t)
    warm_s = time.time() - t0
    t0 = time.time()
    oracle.solve_newton(prob, max_iter=1, beta0=beta)
    step_s = time.time() - t0
    host = "unknown"
    for line in open("/proc/cpuinfo"):
        if line.startswith("model name"):
            host = line.split(":", 1)[1].strip()
            break
    np.savez(os.path.join(OUT, f"{name}.npz"), warm_start_s=np.array(warm_s), warm_assemble_s=np.array(t["assemble_s"]),
             warm_qr_s=np.array(t["solve_s"]), first_newton_step_s=np.array(step_s), threads=np.array(1.0),
             host=np.array(host))
    print(name, "warm start", warm_s, "s, first Newton step", step_s, "s, one core of", host, flush=True)


def pde_residuals(name):
    """The PDE residual of the oracle's stored solutions at the test points (the interior operator,
    plus the nonlinearity where there is one, minus the data), per configuration."""
    out = {}
    for cfg in ("poisson2d", "poisson6d", "heat4d", "reaction2d"):
        g = np.load(os.path.join(OUT, f"{cfg}.npz"))
        prob = wl.config(cfg)
        terms = prob.blocks[0].terms
        r = oracle.apply_operator(prob.W, prob.b, g["beta"], prob.x_test, terms, prob.normalize)
        if prob.nonlin_block == 0:
            u = oracle.evaluate(prob.W, prob.b, g["beta"], prob.x_test, [tuple([0] * prob.d)], prob.normalize)[:, 0]
            r = r + sum(c * u ** k for k, c in enumerate(prob.nonlin_poly))
        r = r - prob.extras["f_test"]
        scale = np.linalg.norm(prob.extras["residual_scale_test"])
        out[f"{cfg}_residual"] = r
        out[f"{cfg}_rel"] = np.array(np.linalg.norm(r) / scale)
        print(cfg, "oracle PDE residual on the test set (relative)", float(out[f"{cfg}_rel"]), flush=True)
    np.savez(os.path.join(OUT, f"{name}.npz"), **out)


HEAT_ALPHAS = [(0, 0, 0, 0), (1, 0, 0, 0), (0, 1, 0, 0), (0, 0, 1, 0), (0, 0, 0, 1)]


def heat4d_eval(name):
    """The oracle's FP64 u, u_x, u_y, u_z, u_t of the stored heat solution at 4096 of the 2^20 query
    points (seeded sample, coordinates rounded to FP32 as the GPU evaluation receives them)."""
    prob = wl.config("heat4d")
    g = np.load(os.path.join(OUT, "heat4d.npz"))
    xq = prob.extras["x_query"]
    idx = np.sort(np.random.default_rng(23).choice(xq.shape[0], 4096, replace=False))
    xr = xq[idx].astype(np.float32).astype(np.float64)
    ref = oracle.evaluate(prob.W, prob.b, g["beta"], xr, HEAT_ALPHAS)
    np.savez(os.path.join(OUT, f"{name}.npz"), idx=idx, ref=ref)
    ex = wl.heat_exact_outputs(xr)
    print(name, "oracle vs exact, rel L2 per output:",
          [float(np.linalg.norm(ref[:, a] - ex[:, a]) / np.linalg.norm(ex[:, a])) for a in range(5)], flush=True)


def sweep(name):
    """All right-hand sides of the sweep from one Householder QR of [A; sqrt(mu) I] (the oracle's
    Tikhonov solve with a matrix right-hand side), u at the test points for each."""
    prob = wl.config(name)
    A, _ = oracle.assemble_system(prob)
    Y = prob.extras["rhs_rows"]
    t0 = time.time()
    B = oracle.tikhonov(A, Y, prob.mu)
    solve_s = time.time() - t0
    U = np.stack([oracle.evaluate(prob.W, prob.b, B[:, s], prob.x_test, [tuple([0] * prob.d)])[:, 0]
                  for s in range(B.shape[1])], axis=1)
    ex = prob.extras["u_test_sweep"]
    err = np.linalg.norm(U - ex, axis=0) / np.linalg.norm(ex, axis=0)
    np.savez(os.path.join(OUT, f"{name}.npz"), u_test=U, err_exact=err, solve_s=np.array(solve_s),
             threads=np.array(oracle.num_threads()))
    print(name, "rel err vs exact: max", err.max(), "median", np.median(err), "QR + solve", solve_s, "s", flush=True)


def bandwidth(name):
    """Loss and L gradient at sigma0 I and at an anisotropic L, and the 80-step AdamW trajectory of
    the scalar bandwidth (lr 0.1, from sigma0), all from the oracle."""
    prob = wl.config(name)
    L0 = prob.extras["L0"]
    La = np.array([[6.0, 0.0], [1.5, 9.0]])
    t0 = time.time()
    loss0, grad0, beta0 = oracle.bandwidth_loss_and_grad(prob, prob.W, L0)
    eval_s = time.time() - t0
    lossa, grada, _ = oracle.bandwidth_loss_and_grad(prob, prob.W, La)
    diag = [k for k, (p, q) in enumerate(oracle.lower_index(prob.d)) if p == q]

    def gfn(sig):
        lo, g, _ = oracle.bandwidth_loss_and_grad(prob, prob.W, sig * np.eye(prob.d))
        return lo, float(g[diag].sum())
    sigs, losses = oracle.adamw_sigma(gfn, prob.extras["sigma0"])
    np.savez(os.path.join(OUT, f"{name}.npz"), loss0=np.array(loss0), grad0=grad0, beta0=beta0, L_aniso=La,
             loss_aniso=np.array(lossa), grad_aniso=grada, adamw_sigma=sigs, adamw_loss=losses,
             eval_s=np.array(eval_s), threads=np.array(oracle.num_threads()))
    print(name, "loss", loss0, "grad", grad0, "adamw: sigma", sigs[-1], "loss", losses[0], "->", losses[-1],
          "eval", eval_s, "s", flush=True)


def varcoef(name):
    """The row-dependent-coefficient solve: beta and u at the test points."""
    prob = wl.config(name)
    t0 = time.time()
    beta = oracle.solve_linear_var(prob)
    solve_s = time.time() - t0
    u = oracle.evaluate(prob.W, prob.b, beta, prob.x_test, [tuple([0] * prob.d)])[:, 0]
    err = oracle.rel_l2(u, prob.u_test)
    np.savez(os.path.join(OUT, f"{name}.npz"), beta=beta, u_test=u, err_exact=np.array(err), solve_s=np.array(solve_s),
             threads=np.array(oracle.num_threads()))
    print(name, "rel err vs exact", err, "solve", solve_s, "s", flush=True)


BURGERS_NEWTON = dict(max_iter=20, tol_du=1e-8, armijo_c=1e-4, max_halvings=10)


def burgers(name):
    """Continuation nu = 1, 0.5, 0.2, 0.1 (Section 2.4), each stage's Newton from the previous
    solution: final beta, u at the test points, and every stage's residual norms."""
    t0 = time.time()
    beta, traces = oracle.continuation(lambda nu: wl.burgers_1d(nu=nu), wl.BURGERS_STAGES, **BURGERS_NEWTON)
    total_s = time.time() - t0
    prob = wl.burgers_1d(nu=wl.BURGERS_STAGES[-1])
    u = oracle.evaluate(prob.W, prob.b, beta, prob.x_test, [(0,)])[:, 0]
    err = oracle.rel_l2(u, prob.u_test)
    iters = np.array([len(t) for t in traces])
    res = np.zeros((len(traces), BURGERS_NEWTON["max_iter"]))
    for k, t in enumerate(traces):
        res[k, :len(t)] = [e["res_norm"] for e in t]
    np.savez(os.path.join(OUT, f"{name}.npz"), beta=beta, u_test=u, err_exact=np.array(err), iters=iters,
             res_norm=res, total_s=np.array(total_s), threads=np.array(oracle.num_threads()))
    print(name, "rel err vs exact", err, "iterations per stage", iters, "total", total_s, "s", flush=True)


def bratu(name):
    """Bratu (lambda = 1) by Newton from the linear warm start, stopped at ||Delta u|| / ||u|| < 1e-8."""
    prob = wl.config(name)
    t0 = time.time()
    beta, trace = oracle.solve_newton_var(prob, max_iter=20, tol_du=1e-8)
    total_s = time.time() - t0
    u = oracle.evaluate(prob.W, prob.b, beta, prob.x_test, [(0, 0)])[:, 0]
    err = oracle.rel_l2(u, prob.u_test)
    np.savez(os.path.join(OUT, f"{name}.npz"), beta=beta, u_test=u, err_exact=np.array(err),
             res_norm=np.array([t["res_norm"] for t in trace]), du_rel=np.array([t["du_rel"] for t in trace]),
             total_s=np.array(total_s), threads=np.array(oracle.num_threads()))
    print(name, "rel err vs exact", err, "steps", len(trace), "total", total_s, "s", flush=True)


KIND = {"poisson2d": linear, "poisson6d": linear, "heat4d": linear, "reaction2d": newton, "inverse3d": inverse,
        "inverse3d_adam": inverse_adam, "reaction2d_timing": reaction2d_timing,
        "pde_residuals": pde_residuals, "heat4d_eval": heat4d_eval,
        "helmholtz_sweep": sweep, "helmholtz_bandwidth": bandwidth,
        "varcoef2d": varcoef, "burgers1d": burgers, "bratu2d": bratu}

if __name__ == "__main__":
    names = sys.argv[1:] or ["poisson2d", "poisson6d"]
    for nm in names:
        t0 = time.time()
        KIND[nm](nm)
        print(nm, "done in", time.time() - t0, "s", flush=True)
