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


if __name__ == "__main__":
    names = sys.argv[1:] or ["poisson2d", "poisson6d"]
    for nm in names:
        t0 = time.time()
        linear(nm)
        print(nm, "done in", time.time() - t0, "s", flush=True)
