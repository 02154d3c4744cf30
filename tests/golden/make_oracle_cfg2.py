"""Writes the oracle results for the 32^3 cube workload (N = 220,256, leaf 64,
eta 2, eps 1e-3, GMRES(50) to 1e-8): tests/golden/oracle_cfg2_k{kappa}.json
and the oracle's solutions in tests/golden/oracle_cfg2_k{kappa}_x.npz.
Calls only the oracle (and the seeded input draw).

Stored per solve: GMRES iterations, relative and absolute residual, the
error against x*, and the oracle solution x as the difference x - x*
quantised to int16 with one scale per column (x is recovered as
x* + scale * q; the quantisation error, at most scale / 2 per entry, is
of the order of 1e-4 of ||x - x*|| in norm, far below the GPU-vs-oracle
differences it is used to measure).  Also stored: the factor error of the oracle factors and
of the same factors rounded to FP32 storage (the floor of the FP32 mode's
factor error), ranks and the oracle's own times (one core).

Usage: python tests/golden/make_oracle_cfg2.py KAPPA NCOLS_PER_SEED SEEDS MAX_ITERS
       (the committed files: 8 8 0,1,2 500 and 16 1 0,1 500)
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


def main(kappa, nrhs, seeds, max_iters, n=32, leaf=64, eps=1e-3):
    here = os.path.dirname(os.path.abspath(__file__))
    tag = f"oracle_cfg2_k{int(kappa)}"
    t0 = time.time()
    d = Discretisation(n, kappa)
    s = Structure(d.mesh.midpoints2(), leaf, 2.0)
    h = HLU(s, d.A, eps)
    t = time.time()
    h.factor()
    t_factor = time.time() - t
    print(f"factor {t_factor:.1f} s", flush=True)
    ranks = h.H.ranks()
    out = dict(n=n, kappa=kappa, eps=eps, leaf=leaf, N=d.N, restart=50, tol=1e-8, max_iters=max_iters,
               factor_error=h.factor_error(), factor_error_fp32_storage=h.factor_error(storage=np.float32),
               max_rank=int(max(ranks)), mean_rank=float(np.mean(ranks)), oracle_factor_s=t_factor,
               oracle_threads=1, solves=[])
    q_all, scale_all = [], []
    for seed in seeds:
        X = exact_solution_cols(d.N, nrhs, seed=seed)
        for c in range(nrhs):
            b = d.A @ X[c]
            t = time.time()
            x, info = gmres(d.A, b, h.solve, restart=50, tol=1e-8, max_iters=max_iters)
            dt = time.time() - t
            diff = x - X[c]
            scale = float(np.abs(diff).max()) / 32767.0 or 1.0
            q = np.round(diff / scale).astype(np.int16)
            q_all.append(q)
            scale_all.append(scale)
            out["solves"].append(dict(seed=seed, col=c, iters=info["iters"], converged=bool(info["converged"]),
                                      relres=float(info["relres"]), abs_res=float(info["abs_res"]),
                                      err=float(np.linalg.norm(diff) / np.linalg.norm(X[c])),
                                      seconds=dt))
            print(f"seed {seed} col {c}: {info['iters']} iters, relres {info['relres']:.2e}, {dt:.1f} s",
                  flush=True)
    out["total_s"] = time.time() - t0
    np.savez_compressed(os.path.join(here, tag + "_x.npz"), q=np.stack(q_all), scale=np.asarray(scale_all),
                        seeds=np.asarray([r["seed"] for r in out["solves"]]),
                        cols=np.asarray([r["col"] for r in out["solves"]]))
    with open(os.path.join(here, tag + ".json"), "w") as f:
        json.dump(out, f, indent=1)
    print(tag, out["factor_error"], out["factor_error_fp32_storage"], [r["iters"] for r in out["solves"]])


if __name__ == "__main__":
    main(float(sys.argv[1]), int(sys.argv[2]), [int(v) for v in sys.argv[3].split(",")], int(sys.argv[4]))
