"""Writes tests/golden/oracle_hinverse_n{n}_k{kappa}_e{eps}.json: the oracle's
Schulz H-inverse (oracle/hinverse.py) on the Kuhn cube, and GMRES(30) to
1e-10 preconditioned by it.  Calls only the oracle (and the seeded input
draw).  Stored: the probed residual after every kept step (probe: N x 8
standard normal from default_rng(12345), cluster order), the steps, the
ranks of B_H, and per right-hand side (x* = exact_solution_cols(N, 3,
seed=1)) the GMRES iterations, relative residual and error against x*.

Usage: python tests/golden/make_oracle_hinverse.py N KAPPA LEAF EPS TOL MAX_ITERS
"""
import json
import os
import sys
import time

os.environ.setdefault("OPENBLAS_NUM_THREADS", "1")
ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

import numpy as np  # noqa: E402

from oracle.assemble import Discretisation  # noqa: E402
from oracle.cluster import Structure  # noqa: E402
from oracle.hinverse import HInverse  # noqa: E402
from oracle.krylov import gmres  # noqa: E402
from paper_2211_11303_amd.inputs import exact_solution_cols  # noqa: E402


def main(n, kappa, leaf, eps, tol, max_iters):
    d = Discretisation(n, kappa)
    s = Structure(d.mesh.midpoints2(), leaf, 2.0)
    h = HInverse(s, d.A, eps)
    t = time.time()
    rho = h.residual()
    h.history = [rho]
    for k in range(max_iters):   # HInverse.compute, with progress lines
        if rho <= tol:
            break
        Xn = h.step(h.X)
        rn = h.residual(Xn)
        print(f"step {k + 1}: rho {rn:.3e} ({time.time() - t:.0f} s)", flush=True)
        if rn >= rho:
            break
        h.X, rho = Xn, rn
        h.history.append(rho)
    t_inv = time.time() - t
    ranks = h.X.ranks()
    out = dict(n=n, kappa=kappa, leaf=leaf, eps=eps, tol=tol, max_iters=max_iters, N=d.N, steps=h.iterations,
               history=h.history, max_rank=int(max(ranks) if ranks else 0),
               mean_rank=float(np.mean(ranks)) if ranks else 0.0, oracle_seconds=t_inv, solves=[])
    X = exact_solution_cols(d.N, 3, seed=1)
    for c in range(3):
        b = d.A @ X[c]
        x, info = gmres(d.A, b, h.solve, restart=30, tol=1e-10, max_iters=500)
        out["solves"].append(dict(col=c, iters=info["iters"], converged=bool(info["converged"]),
                                  relres=float(info["relres"]),
                                  err=float(np.linalg.norm(x - X[c]) / np.linalg.norm(X[c]))))
    path = os.path.join(os.path.dirname(os.path.abspath(__file__)),
                        f"oracle_hinverse_n{n}_k{int(kappa)}_e{eps:.0e}.json")
    with open(path, "w") as f:
        json.dump(out, f, indent=1)
    print(path, h.iterations, h.history[-1], [r["iters"] for r in out["solves"]])


if __name__ == "__main__":
    main(int(sys.argv[1]), float(sys.argv[2]), int(sys.argv[3]), float(sys.argv[4]), float(sys.argv[5]),
         int(sys.argv[6]))
