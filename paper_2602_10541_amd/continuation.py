"""Continuation (homotopy) for the Newton solver, Section 2.4: a sequence of problems in a
parameter (the Burgers viscosity nu = 1 -> 0.5 -> 0.2 -> 0.1), each solved by
``flsq_solve_newton_var`` from the previous stage's coefficients; the first stage starts from
its linear warm start."""
from __future__ import annotations

from . import fastlsq as fl


def newton_opts(mu, max_iter=20, armijo_c=1e-4, max_halvings=10, max_refine=30, refine_tol=1e-12, tol_dbeta=0.0,
                warm_start=True):
    return fl.flsq_newton_opts(fl.solve_opts(mu, fl.PREC_FP64, max_refine, refine_tol), float(tol_dbeta),
                               int(max_iter), float(armijo_c), int(max_halvings), 1 if warm_start else 0)


def solve_continuation(ctx, stages, make_device_problem, beta, tol_du=1e-8, **opts_kw):
    """stages: parameter values in order; make_device_problem(p) -> (DeviceVarProblem, nonlin_block,
    poly, adv, mu).  beta (device, n_feat) receives the last stage's solution.  Returns the
    Newton traces of the stages (lists of per-step dicts) and their statuses."""
    traces, statuses = [], []
    for k, p in enumerate(stages):
        dp, nl_block, poly, adv, mu = make_device_problem(p)
        opts = newton_opts(mu, warm_start=(k == 0), **opts_kw)
        st, tr = fl.flsq_solve_newton_var(ctx, dp.basis, dp.rows, nl_block, poly, adv, opts, tol_du, beta)
        traces.append(tr.as_list())
        statuses.append(st)
    return traces, statuses
