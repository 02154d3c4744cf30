"""GPU tests of the device-side failure paths, each forced from the host so
that every kernel still exits normally.

* A truncation whose eps-rank reaches the block's 64-column capacity while
  parts remain (16^3, leaf 64, kappa 30 = the paper's kappa 900, eps 1e-3:
  the oracle's ranks reach 73) ends with HLU_ERR_RANK_OVERFLOW.
* A persistent solve whose waits are given a zero time limit (the
  HLU_DEBUG_SOLVE_WAIT_US switch) reports HLU_ERR_DEVICE through
  hlu_sync_status and gmres_solve, and the next solve with the normal limit
  is correct again.
* Determinism: factor and solve twice, identical bytes."""
import os
import time

import numpy as np
import pytest

from gpu_util import oracle_problem

pytestmark = pytest.mark.gpu


def _lib():
    from paper_2211_11303_amd import _lib as L, hlu, inputs
    return L, hlu, inputs


def test_rank_overflow_is_reported(gpu):
    L, hlu, _ = _lib()
    print("case: 16^3 leaf 64 kappa 30 eps 1e-3 fp64", flush=True)
    rp, ci, va, mid = hlu.hlu_kuhn_assemble(16, 30.0)
    H = hlu.HLU(rp, ci, va, mid, 2.0, 64)
    t = time.time()
    with pytest.raises(L.HluError) as e:
        H.hlu_factor(1e-3, prec="fp64")
    assert e.value.status == L.STATUS_CODES["HLU_ERR_RANK_OVERFLOW"]
    assert time.time() - t < 60.0
    st = H.hlu_get_stats()
    assert st["capped_blocks"] > 0 and st["max_rank"] <= 64, st
    # the factor is kept at capacity and usable
    H2 = H.hlu_factor(1e-3, prec="fp64", allow_overflow=True)
    import torch
    b = torch.ones((1, H.n), dtype=torch.float64, device="cuda")
    x = H2.hlu_solve(b)
    torch.cuda.synchronize()
    assert torch.isfinite(x).all()


def test_solve_wait_timeout_is_reported(gpu):
    import torch
    L, hlu, inputs = _lib()
    n, kappa, leaf = 8, 4.0, 32
    rp, ci, va, mid = hlu.hlu_kuhn_assemble(n, kappa)
    A = hlu.SpMat(rp, ci, va)
    H = hlu.HLU(rp, ci, va, mid, 2.0, leaf).hlu_factor(1e-4, prec="fp64")
    d, _ = oracle_problem(n, kappa, leaf)
    X = inputs.exact_solution_cols(A.n, 4, seed=5)
    B = torch.tensor(np.stack([d.A @ x for x in X]), device="cuda")
    x_ref = H.hlu_solve(B).clone()
    H.hlu_sync_status()
    print("case: 8^3 solve with a zero wait limit", flush=True)
    os.environ["HLU_DEBUG_SOLVE_WAIT_US"] = "0"
    try:
        H.hlu_solve(B)
        with pytest.raises(L.HluError) as e:
            H.hlu_sync_status()
        assert e.value.status == L.STATUS_CODES["HLU_ERR_DEVICE"]
        with pytest.raises(L.HluError) as e:
            hlu.gmres_solve(A, B, H, restart=20, tol=1e-8)
        assert e.value.status == L.STATUS_CODES["HLU_ERR_DEVICE"]
    finally:
        del os.environ["HLU_DEBUG_SOLVE_WAIT_US"]
    H.hlu_sync_status()   # the report was consumed
    x2 = H.hlu_solve(B)
    H.hlu_sync_status()
    assert torch.equal(x2, x_ref)


def test_factor_and_solve_are_deterministic(gpu):
    import torch
    _, hlu, inputs = _lib()
    n, kappa, leaf = 16, 8.0, 64
    rp, ci, va, mid = hlu.hlu_kuhn_assemble(n, kappa)
    X = torch.tensor(inputs.exact_solution_cols(len(rp) - 1, 8, seed=2), device="cuda")
    for prec in ("fp64", "fp32"):
        out = []
        for _ in range(2):
            H = hlu.HLU(rp, ci, va, mid, 2.0, leaf).hlu_factor(1e-4, prec=prec)
            arena = H.work.clone()
            x1 = H.hlu_solve(X).clone()
            x2 = H.hlu_solve(X).clone()
            H.hlu_sync_status()
            out.append((arena, x1, x2, H.hlu_get_ranks()))
        (a0, x10, x20, r0), (a1, x11, x21, r1) = out
        assert np.array_equal(r0, r1), prec
        assert torch.equal(a0, a1), prec
        assert torch.equal(x10, x20) and torch.equal(x10, x11) and torch.equal(x20, x21), prec
