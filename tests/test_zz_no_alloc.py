"""gmres_solve_static (no device allocation inside the call) against
gmres_solve with a caller workspace, through the C ABI: two calls in a row,
the second on a smaller problem, each to the GMRES parity bar (same
iteration counts, same solution up to rounding); sizes beyond the static
workspace are rejected on the host."""
import numpy as np
import pytest

pytestmark = pytest.mark.gpu


def _case(n, kappa, leaf, eps, nrhs, seed):
    import torch
    from paper_2211_11303_amd import hlu, inputs
    rp, ci, va, mid = hlu.hlu_kuhn_assemble(n, kappa)
    A = hlu.SpMat(rp, ci, va)
    H = hlu.HLU(rp, ci, va, mid, 2.0, leaf).hlu_factor(eps, prec="fp32")
    X = torch.tensor(inputs.exact_solution_cols(A.n, nrhs, seed=seed), device="cuda")
    B = A.hlu_spmv(X)
    return A, H, B


def test_static_gmres_matches_workspace_gmres(gpu):
    import torch
    from paper_2211_11303_amd import _lib as L, hlu
    assert hlu.gmres_static_max_bytes() == 64 << 20
    for (n, kappa, leaf, eps, nrhs, seed) in ((12, 6.0, 64, 1e-3, 4, 1), (8, 3.0, 32, 1e-4, 2, 2)):
        print(f"case: n={n} nrhs={nrhs}", flush=True)
        A, H, B = _case(n, kappa, leaf, eps, nrhs, seed)
        assert hlu.gmres_workspace_bytes(A.n, nrhs, 30) <= hlu.gmres_static_max_bytes()
        x_ref, info_ref = hlu.gmres_solve(A, B, H, restart=30, tol=1e-8)
        x, info = hlu.gmres_solve_static(A, B, H, restart=30, tol=1e-8)
        torch.cuda.synchronize()
        for a, b in zip(info, info_ref):
            assert a["converged"] and a["iters"] == b["iters"], (info, info_ref)
            assert abs(a["relres"] - b["relres"]) <= 1e-12
        assert torch.allclose(x, x_ref, rtol=0, atol=1e-13 * float(x_ref.abs().max()))
    # too large for the static workspace: rejected before any device work
    rp, ci, va, _ = hlu.hlu_kuhn_assemble(24, 4.0)
    big = hlu.SpMat(rp, ci, va)
    Bb = torch.ones((8, big.n), dtype=torch.float64, device="cuda")
    with pytest.raises(L.HluError) as e:
        hlu.gmres_solve_static(big, Bb, None, restart=50, tol=1e-8)
    assert e.value.status == L.STATUS_CODES["HLU_ERR_OUT_OF_MEMORY"]
