"""Batched factorisation, solve and GMRES (hlu_batch_*) against the same
problems run one by one, and members against the oracle.

A batch runs every member's tasks in the member's own order with the same
kernels, so its results must equal the one-by-one results up to the
summation order of the GMRES dot products (identical here: the per-segment
partition is the same); the bar is 1e-13 relative for factors and solves and
equal iteration counts for GMRES.  Oracle parity of the members, FP64 and
FP32: factor error within 2x the oracle's plus the Gram-truncation floor
u/eps (FP32: plus the FP32 rounding terms of gpu_util.fp32_factor_bound),
GMRES iterations within +-1."""
import numpy as np
import pytest

from gpu_util import fp32_factor_bound, gpu_factor_error, oracle_factor, oracle_problem, oracle_solve

pytestmark = pytest.mark.gpu

# (n, kappa, leaf): two members share a mesh (and so a structure), leaves differ
MEMBERS = [(4, 2.0, 32), (5, 3.0, 20), (4, 5.0, 32), (6, 1.5, 48)]


def _members(share=True):
    from paper_2211_11303_amd import hlu
    out, protos = [], {}
    for n, kappa, leaf in MEMBERS:
        rp, ci, va, mid = hlu.hlu_kuhn_assemble(n, kappa)
        A = hlu.SpMat(rp, ci, va)
        key = (n, leaf)
        if share and key in protos:
            H = hlu.HLU(rp, ci, va, share=protos[key])
        else:
            H = hlu.HLU(rp, ci, va, mid, 2.0, leaf)
            protos[key] = H
        out.append((A, H))
    return out


def _rhs(batch, members, nrhs, seed):
    import torch
    from paper_2211_11303_amd import inputs
    xs = [torch.tensor(inputs.exact_solution_cols(A.n, nrhs, seed=seed + p), device="cuda")
          for p, (A, _) in enumerate(members)]
    bs = [A.hlu_spmv(x) for (A, _), x in zip(members, xs)]
    return xs, bs, batch.stack(bs)


@pytest.mark.parametrize("prec", ["fp64", "fp32", "fp32-acc64"])
def test_batch_equals_one_by_one(gpu, prec):
    import torch
    from paper_2211_11303_amd import hlu
    eps = 1e-6 if prec == "fp64" else 1e-4
    single = _members(share=False)
    for _, H in single:
        H.hlu_factor(eps, prec=prec)
    batched = _members(share=True)
    B = hlu.HLUBatch([H for _, H in batched], eps, prec=prec, max_rhs=3)
    assert B.factor_waves == max(H.hlu_get_stats()["factor_waves"] for _, H in single)
    B.hlu_factor_batch()
    xs, bs, bstack = _rhs(B, batched, 3, seed=20)
    # members used on their own after the batch factorisation
    for (A, Hs), (_, Hb), b in zip(single, batched, bs):
        zs = Hs.hlu_solve(b)
        zb = Hb.hlu_solve(b)
        torch.cuda.synchronize()
        assert (zs - zb).norm() <= 1e-13 * zs.norm(), (A.n, (zs - zb).norm().item())
    # one persistent launch for all members
    z = B.unstack(B.hlu_solve_batch(bstack))
    for (A, Hs), b, zp in zip(single, bs, z):
        zs = Hs.hlu_solve(b)
        assert (zs - zp).norm() <= 1e-13 * zs.norm(), (A.n, (zs - zp).norm().item())
    # GMRES for all members at once
    xb, infos = B.gmres_solve_batch(bstack, restart=30, tol=1e-10)
    xb = B.unstack(xb)
    for p, ((A, Hs), b) in enumerate(zip(single, bs)):
        xs_p, inf_s = hlu.gmres_solve(A, b, Hs, restart=30, tol=1e-10)
        for c in range(3):
            assert infos[p][c]["converged"] and infos[p][c]["iters"] == inf_s[c]["iters"], (p, c, infos[p][c],
                                                                                            inf_s[c])
        assert (xb[p] - xs_p).norm() <= 1e-10 * xs_p.norm()


@pytest.mark.parametrize("prec,eps", [("fp64", 1e-6), ("fp32", 1e-4)])
def test_batch_members_against_oracle(gpu, prec, eps):
    import torch
    from paper_2211_11303_amd import hlu
    batched = _members(share=True)
    B = hlu.HLUBatch([H for _, H in batched], eps, prec=prec, max_rhs=1).hlu_factor_batch()
    xs, bs, bstack = _rhs(B, batched, 1, seed=3)
    xb, infos = B.gmres_solve_batch(bstack, restart=30, tol=1e-10)
    for p, (n, kappa, leaf) in enumerate(MEMBERS):
        A, H = batched[p]
        d, s = oracle_problem(n, kappa, leaf)
        e_gpu = gpu_factor_error(H, d.A, s.perm)
        o = oracle_factor(n, kappa, leaf, eps)
        e_ora = o.factor_error()
        # the Gram-based truncation reconstructs a kept singular triplet of
        # size ~eps sigma_1 with absolute error ~u sigma_1^2 / (eps sigma_1)
        floor = np.finfo(np.float64).eps / eps
        bar = (2 * e_ora + floor if prec == "fp64"
               else fp32_factor_bound(e_ora, o.factor_error(storage=np.float32), leaf) + floor)
        assert e_gpu <= bar, (p, e_gpu, e_ora, bar)
        _, io = oracle_solve(n, kappa, leaf, eps, bs[p].cpu().numpy()[0], 30, 1e-10)
        assert abs(infos[p][0]["iters"] - io["iters"]) <= 1, (p, infos[p][0], io)
        xp = B.unstack(xb)[p]
        rel = np.linalg.norm(d.A @ xp.cpu().numpy()[0] - bs[p].cpu().numpy()[0]) / np.linalg.norm(
            bs[p].cpu().numpy()[0])
        assert rel <= 1e-10


def test_batch_state_rules(gpu):
    import torch
    from paper_2211_11303_amd import hlu, _lib
    batched = _members(share=True)
    B = hlu.HLUBatch([H for _, H in batched], 1e-6, prec="fp64", max_rhs=2)
    H0 = batched[0][1]
    # a member's workspace is the batch's
    with pytest.raises(_lib.HluError) as e:
        H0.hlu_bind_workspace(1 << 20)
    assert e.value.status == _lib.STATUS_CODES["HLU_ERR_STATE"]
    # solve before factor
    xs, bs, bstack = _rhs(B, batched, 1, seed=0)
    B.hlu_batch_bind_workspace()
    with pytest.raises(_lib.HluError) as e:
        B.hlu_solve_batch(bstack)
    assert e.value.status == _lib.STATUS_CODES["HLU_ERR_STATE"]
    B.hlu_factor_batch()
    # too many columns
    with pytest.raises(_lib.HluError) as e:
        B.hlu_solve_batch(torch.cat([bstack] * 3))
    assert e.value.status == _lib.STATUS_CODES["HLU_ERR_INVALID_ARG"]
    # a member destroyed while in the batch makes it unusable
    import ctypes
    lib = _lib.lib()
    lib.hlu_destroy(batched[1][1].handle)
    batched[1][1].handle = None
    with pytest.raises(_lib.HluError) as e:
        B.hlu_solve_batch(bstack)
    assert e.value.status == _lib.STATUS_CODES["HLU_ERR_STATE"]
