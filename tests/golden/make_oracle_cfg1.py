"""Writes tests/golden/oracle_cfg1_k{kappa}_e{eps}.json: oracle results for
the 16^3 cube workload (leaf 64, eta 2, 8 right-hand sides per seed,
GMRES(50) to 1e-8), including the factor error of the oracle factors
rounded to FP32 storage (the rounding floor of the FP32 mode).  Calls only
the oracle (and the seeded input draw).

Usage: python tests/golden/make_oracle_cfg1.py KAPPA EPS
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
from oracle.hmatrix import HLU  # noqa: E402
from oracle.krylov import gmres  # noqa: E402
from paper_2211_11303_amd.inputs import exact_solution_cols  # noqa: E402


def main(kappa, eps, n=16, leaf=64, seeds=(0, 1, 2), nrhs=8):
    t0 = time.time()
    d = Discretisation(n, kappa)
    s = Structure(d.mesh.midpoints2(), leaf, 2.0)
    h = HLU(s, d.A, eps)
    t = time.time()
    h.factor()
    t_factor = time.time() - t
    ranks = h.H.ranks()
    out = dict(n=n, kappa=kappa, eps=eps, leaf=leaf, N=d.N, factor_error=h.factor_error(),
               factor_error_fp32_storage=h.factor_error(storage=np.float32),
               max_rank=int(max(ranks)), mean_rank=float(np.mean(ranks)), oracle_factor_s=t_factor,
               truncations=h.trunc.count, solves=[])
    for seed in seeds:
        X = exact_solution_cols(d.N, nrhs, seed=seed)
        for c in range(nrhs):
            b = d.A @ X[c]
            t = time.time()
            x, info = gmres(d.A, b, h.solve, restart=50, tol=1e-8, max_iters=500)
            out["solves"].append(dict(seed=seed, col=c, iters=info["iters"], converged=bool(info["converged"]),
                                      relres=float(info["relres"]), abs_res=float(info["abs_res"]),
                                      err=float(np.linalg.norm(x - X[c]) / np.linalg.norm(X[c])),
                                      seconds=time.time() - t))
    out["total_s"] = time.time() - t0
    path = os.path.join(os.path.dirname(os.path.abspath(__file__)),
                        f"oracle_cfg1_k{int(kappa)}_e{eps:.0e}.json")
    with open(path, "w") as f:
        json.dump(out, f, indent=1)
    print(path, out["factor_error"], [s_["iters"] for s_ in out["solves"]])


if __name__ == "__main__":
    main(float(sys.argv[1]), float(sys.argv[2]))
