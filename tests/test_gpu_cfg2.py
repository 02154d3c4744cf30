"""32^3 cube workload (N = 220,256, leaf 64, eta 2, eps 1e-3, GMRES(50) to
1e-8) on the GPU, FP64 and FP32 H-LU, against the oracle's stored results
(tests/golden/oracle_cfg2_k*.json and *_x.npz, written by
tests/golden/make_oracle_cfg2.py, which calls only the oracle).

Bars:
  - factor error: FP64 within 2x the oracle's; FP32 within
    gpu_util.fp32_factor_bound (2x the oracle's plus the FP32 rounding terms
    derived from the oracle's own factors rounded to FP32);
  - kappa = 8, all 24 right-hand sides: GMRES iterations within +-1 of the
    oracle's, true relative residual <= 1e-8, and the distance to the
    oracle's solution ||x - x_oracle|| <= 3 max(e_or, a res) (relative),
    e_or = ||x_oracle - x*||/||x*||, a = e_or / (the oracle's final relative
    residual) the system's amplification of a residual, res the GPU's final
    relative residual: the GPU's own error is bounded like the oracle's
    through its residual, taken as at most 2x, and the distance by the sum
    of the two errors;
  - kappa = 16 lies 0.24 % below the cavity eigenvalue 26 pi^2, where GMRES
    iteration counts change by hundreds under perturbations of the factor far
    below its own error (the oracle needs 497 and 500 iterations, the GPU
    factors, whose errors are smaller, 100-300).  There the bar is the factor
    error, convergence within the oracle's iteration count and the same
    solution-distance bar as above (parity of the count itself unpinned)."""
import json
import os

import numpy as np
import pytest

from gpu_util import fp32_factor_bound, gpu_factor_error

pytestmark = pytest.mark.gpu
GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def _golden(kappa):
    g = json.load(open(os.path.join(GOLDEN, f"oracle_cfg2_k{int(kappa)}.json")))
    z = np.load(os.path.join(GOLDEN, f"oracle_cfg2_k{int(kappa)}_x.npz"))
    return g, z


@pytest.fixture(scope="module")
def proto32():
    from paper_2211_11303_amd import hlu
    rp, ci, va, mid = hlu.hlu_kuhn_assemble(32, 8.0)
    return hlu.HLU(rp, ci, va, mid, 2.0, 64)


def _run(proto, kappa, prec, iters_bar):
    import scipy.sparse as sp
    import torch
    from paper_2211_11303_amd import hlu, inputs
    g, z = _golden(kappa)
    rp, ci, va, _ = hlu.hlu_kuhn_assemble(32, kappa)
    A = hlu.SpMat(rp, ci, va)
    Acsr = sp.csr_matrix((va, ci, rp), shape=(A.n, A.n))
    H = hlu.HLU(rp, ci, va, share=proto).hlu_factor(1e-3, prec=prec)
    e = gpu_factor_error(H, Acsr, H.hlu_export_structure()["perm"])
    bar = 2 * g["factor_error"] if prec == "fp64" else fp32_factor_bound(g["factor_error"],
                                                                        g["factor_error_fp32_storage"], 64)
    print(f"kappa {kappa:g} {prec}: factor error {e:.3e} (oracle {g['factor_error']:.3e}, bar {bar:.3e})",
          flush=True)
    assert e <= bar, (e, bar)
    from oracle.assemble import Discretisation
    Aor = Discretisation(32, kappa).A   # the oracle's matrix: its right-hand sides, bit for bit
    seeds = sorted({int(v) for v in z["seeds"]})
    ncol = int(max(z["cols"])) + 1
    for seed in seeds:
        X = inputs.exact_solution_cols(A.n, ncol, seed=seed)
        B = (Aor @ X.T).T.copy()
        x, infos = hlu.gmres_solve(A, torch.tensor(B, device="cuda"), H, restart=50, tol=1e-8, max_iters=600)
        xg = x.cpu().numpy()
        for c in range(ncol):
            k = int(np.flatnonzero((z["seeds"] == seed) & (z["cols"] == c))[0])
            ref = g["solves"][k]
            xo = X[c] + z["scale"][k] * z["q"][k].astype(np.float64)
            relres = np.linalg.norm(Acsr @ xg[c] - B[c]) / np.linalg.norm(B[c])
            d_or = np.linalg.norm(xg[c] - xo) / np.linalg.norm(xo)
            print(f"  seed {seed} col {c}: iters {infos[c]['iters']} (oracle {ref['iters']}), relres "
                  f"{relres:.2e}, |x - x_oracle|/|x_oracle| {d_or:.2e} (oracle err {ref['err']:.2e})", flush=True)
            assert infos[c]["converged"] and relres <= 1e-8
            iters_bar(infos[c]["iters"], ref["iters"])
            amp = ref["err"] / max(ref["relres"], 1e-300)   # residual amplification of this system
            assert d_or <= 3 * max(ref["err"], amp * relres), (seed, c, d_or, ref["err"], relres)
    del H


@pytest.mark.parametrize("prec", ["fp64", "fp32"])
def test_cfg2_kappa8_against_oracle(gpu, proto32, prec):
    def bar(it, it_or):
        assert abs(it - it_or) <= 1, (it, it_or)
    _run(proto32, 8.0, prec, bar)


@pytest.mark.parametrize("prec", ["fp64", "fp32"])
def test_cfg2_kappa16_near_resonance(gpu, proto32, prec):
    def bar(it, it_or):
        assert it <= it_or, (it, it_or)
    _run(proto32, 16.0, prec, bar)
