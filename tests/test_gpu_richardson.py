"""Preconditioned Richardson iteration of Algorithm 1, steps III-IV
(hlu_richardson) against the oracle's (oracle.krylov.richardson) with the
oracle's H-LU of the same eps and leaf, on the same right-hand sides.

Bars: corrections applied within +-1 of the oracle's per column; the
paper's stopping order (the correction after the test is still applied,
so the final error is below the last measured one); final relative
residual within 10x the oracle's or below 1e-12 relative."""
import numpy as np
import pytest

from gpu_util import oracle_factor, oracle_problem

pytestmark = pytest.mark.gpu


@pytest.mark.parametrize("n,kappa,leaf,eps,tol,prec", [(4, 2.0, 32, 1e-6, 1e-10, "fp64"),
                                                        (8, 4.0, 64, 1e-3, 1e-8, "fp64"),
                                                        (8, 4.0, 64, 1e-3, 1e-8, "fp32")])
def test_richardson_against_oracle(gpu, n, kappa, leaf, eps, tol, prec):
    import torch
    from oracle.krylov import richardson
    from paper_2211_11303_amd import hlu, inputs
    d, s = oracle_problem(n, kappa, leaf)
    o = oracle_factor(n, kappa, leaf, eps)
    rp, ci, va, mid = hlu.hlu_kuhn_assemble(n, kappa)
    A = hlu.SpMat(rp, ci, va)
    H = hlu.HLU(rp, ci, va, mid, 2.0, leaf).hlu_factor(eps, prec=prec)
    X = inputs.exact_solution_cols(A.n, 3, seed=2)
    B = (d.A @ X.T).T.copy()
    x, infos = hlu.hlu_richardson(A, torch.tensor(B, device="cuda"), H, tol=tol, max_iters=200)
    xg = x.cpu().numpy()
    for c in range(3):
        xo, io = richardson(d.A, B[c], o.solve, tol=tol, max_iters=200)
        rel = np.linalg.norm(d.A @ xg[c] - B[c]) / np.linalg.norm(B[c])
        print(f"n={n} {prec} col {c}: corrections {infos[c]['iters']} (oracle {io['iters']}), relres {rel:.2e} "
              f"(oracle {io['relres']:.2e})", flush=True)
        assert infos[c]["converged"]
        assert abs(infos[c]["iters"] - io["iters"]) <= 1, (c, infos[c], io)
        assert abs(infos[c]["relres"] - rel) <= 1e-12 + 1e-6 * rel
        assert rel <= max(10 * io["relres"], 1e-12), (c, rel, io["relres"])


def test_richardson_with_schulz_inverse(gpu):
    """Algorithm 1 with B_H (the paper's other preconditioner) in place of
    the H-LU: converges to the same tolerance."""
    import torch
    from paper_2211_11303_amd import hlu, inputs
    d, s = oracle_problem(4, 2.0, 32)
    rp, ci, va, mid = hlu.hlu_kuhn_assemble(4, 2.0)
    A = hlu.SpMat(rp, ci, va)
    H = hlu.HLU(rp, ci, va, mid, 2.0, 32)
    Om = np.random.default_rng(12345).standard_normal((A.n, 8))
    v = np.empty_like(Om)
    v[s.perm] = Om
    info = H.hlu_inverse(torch.tensor(v.T.copy(), device="cuda"), 1e-8, tol=1e-9, max_iters=60)
    assert info["residual"] < 1e-3
    X = inputs.exact_solution_cols(A.n, 2, seed=4)
    B = torch.tensor((d.A @ X.T).T.copy(), device="cuda")
    x, infos = hlu.hlu_richardson(A, B, H, tol=1e-10, max_iters=100)
    for c in range(2):
        assert infos[c]["converged"] and infos[c]["relres"] <= 1e-10
