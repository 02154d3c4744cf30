"""GPU parity tests: the HIP path through the C ABI against the oracle.

Tolerances: SpMV 1e-13 relative (FP64, summation order only); factor error
within 2x the oracle's plus 1e-12 (FP64) or within
gpu_util.fp32_factor_bound (FP32: 2x the oracle's plus the FP32 rounding
terms derived from the oracle's factors rounded to FP32); GMRES iterations
within +-1 of the oracle in every precision and final relative residual
<= tol."""
import numpy as np
import pytest

from gpu_util import fp32_factor_bound, gpu_factor_error, oracle_factor, oracle_problem, oracle_solve

pytestmark = pytest.mark.gpu


def _lib():
    from paper_2211_11303_amd import hlu, inputs
    return hlu, inputs


def _setup(n, kappa, leaf):
    hlu, _ = _lib()
    rp, ci, va, mid = hlu.hlu_kuhn_assemble(n, kappa)
    return hlu.SpMat(rp, ci, va), (rp, ci, va, mid)


@pytest.mark.parametrize("n,nrhs", [(4, 1), (4, 3), (8, 5), (16, 8)])
def test_spmv(gpu, n, nrhs):
    import torch
    hlu, inputs = _lib()
    A, _ = _setup(n, 2.0, 32)
    d, _ = oracle_problem(n, 2.0, 32)
    X = inputs.exact_solution_cols(A.n, nrhs, seed=3)
    Y = A.hlu_spmv(torch.tensor(X, device="cuda")).cpu().numpy()
    ref = (d.A @ X.T).T
    assert np.abs(Y - ref).max() <= 1e-13 * np.abs(ref).max()
    # alpha / beta
    Y2 = torch.tensor(X, device="cuda")
    A.hlu_spmv(torch.tensor(X, device="cuda"), Y2, alpha=2.0, beta=-1.0)
    assert np.abs(Y2.cpu().numpy() - (2 * ref - X)).max() <= 1e-13 * np.abs(ref).max()


@pytest.mark.parametrize("prec", ["fp64", "fp32", "fp32-acc64"])
def test_cfg0_parity(gpu, prec):
    """4^3 cubes, kappa 2, leaf 32, eps 1e-6, GMRES(30) to 1e-10, seeds 0..9."""
    import torch
    hlu, inputs = _lib()
    n, kappa, leaf, eps = 4, 2.0, 32, 1e-6
    A, (rp, ci, va, mid) = _setup(n, kappa, leaf)
    H = hlu.HLU(rp, ci, va, mid, 2.0, leaf).hlu_factor(eps, prec=prec)
    d, s = oracle_problem(n, kappa, leaf)
    o = oracle_factor(n, kappa, leaf, eps)
    e_gpu = gpu_factor_error(H, d.A, s.perm)
    e_or = o.factor_error()
    bar = 2 * e_or + 1e-12 if prec == "fp64" else fp32_factor_bound(e_or, o.factor_error(storage=np.float32), leaf)
    assert e_gpu <= bar, (e_gpu, e_or, bar)
    for seed in range(10):
        xs = inputs.exact_solution_cols(A.n, 1, seed=seed)[0]
        b = d.A @ xs
        x, info = hlu.gmres_solve(A, torch.tensor(b, device="cuda").reshape(1, -1), H, restart=30, tol=1e-10)
        xo, io = oracle_solve(n, kappa, leaf, eps, b, 30, 1e-10)
        xg = x.cpu().numpy()[0]
        relres = np.linalg.norm(d.A @ xg - b) / np.linalg.norm(b)
        assert info[0]["converged"] and relres <= 1e-10
        assert abs(info[0]["iters"] - io["iters"]) <= 1, (seed, info, io)
        assert abs(info[0]["relres"] - relres) <= 1e-12


def test_untruncated_is_exact(gpu):
    """eps = 0: the factors reproduce P A P^T to the Gram truncation floor."""
    hlu, _ = _lib()
    A, (rp, ci, va, mid) = _setup(4, 2.0, 32)
    H = hlu.HLU(rp, ci, va, mid, 2.0, 32).hlu_factor(0.0, prec="fp64")
    d, s = oracle_problem(4, 2.0, 32)
    assert gpu_factor_error(H, d.A, s.perm) <= 1e-9
    # untruncated unpivoted H-LU = dense unpivoted LU of P A P^T: same pivots
    from oracle.hmatrix import getrf_nopiv
    Ap = d.A.toarray()[np.ix_(s.perm, s.perm)]
    piv = np.abs(np.diag(getrf_nopiv(Ap)))
    st = H.hlu_get_stats()
    assert abs(st["min_abs_pivot"] - piv.min()) <= 1e-9 * piv.max()
    assert abs(st["max_abs_pivot"] - piv.max()) <= 1e-9 * piv.max()


@pytest.mark.parametrize("n,leaf,eps", [(5, 20, 1e-4), (4, 8, 1e-4), (3, 4, 1e-3)])
def test_all_product_cases(gpu, n, leaf, eps):
    """Small leaves exercise every case of the H-product recursion and the
    admissible blocks that hold matrix entries."""
    hlu, _ = _lib()
    A, (rp, ci, va, mid) = _setup(n, 2.0, leaf)
    H = hlu.HLU(rp, ci, va, mid, 2.0, leaf).hlu_factor(eps, prec="fp64")
    d, s = oracle_problem(n, 2.0, leaf)
    e_gpu = gpu_factor_error(H, d.A, s.perm)
    e_or = oracle_factor(n, 2.0, leaf, eps).factor_error()
    assert e_gpu <= 2 * e_or + 1e-12, (e_gpu, e_or)


def test_solve_inverts_apply(gpu):
    import torch
    hlu, inputs = _lib()
    A, (rp, ci, va, mid) = _setup(8, 4.0, 64)
    H = hlu.HLU(rp, ci, va, mid, 2.0, 64).hlu_factor(1e-4, prec="fp64")
    for nrhs in (1, 7, 33):        # 33 > the solve plan's column capacity
        y = torch.tensor(inputs.exact_solution_cols(A.n, nrhs, seed=nrhs), device="cuda")
        z = H.hlu_solve(H.hlu_apply_lu(y))
        assert (z - y).norm() <= 1e-10 * y.norm()
        # in place: x aliases b
        w = H.hlu_apply_lu(y)
        H.hlu_solve(w, w)
        assert (w - y).norm() <= 1e-10 * y.norm()


@pytest.mark.parametrize("prec,eps", [("fp64", 1e-4), ("fp32", 1e-3)])
def test_n8_factor_and_gmres(gpu, prec, eps):
    import torch
    hlu, inputs = _lib()
    n, kappa, leaf = 8, 8.0, 64
    A, (rp, ci, va, mid) = _setup(n, kappa, leaf)
    H = hlu.HLU(rp, ci, va, mid, 2.0, leaf).hlu_factor(eps, prec=prec)
    d, s = oracle_problem(n, kappa, leaf)
    e_gpu = gpu_factor_error(H, d.A, s.perm)
    o = oracle_factor(n, kappa, leaf, eps)
    e_or = o.factor_error()
    bar = 2 * e_or + 1e-12 if prec == "fp64" else fp32_factor_bound(e_or, o.factor_error(storage=np.float32), leaf)
    assert e_gpu <= bar, (e_gpu, e_or, bar)
    X = inputs.exact_solution_cols(A.n, 4, seed=1)
    B = (d.A @ X.T).T.copy()
    x, infos = hlu.gmres_solve(A, torch.tensor(B, device="cuda"), H, restart=50, tol=1e-8)
    xg = x.cpu().numpy()
    for c in range(4):
        relres = np.linalg.norm(d.A @ xg[c] - B[c]) / np.linalg.norm(B[c])
        assert infos[c]["converged"] and relres <= 1e-8
        xo, io = oracle_solve(n, kappa, leaf, eps, B[c], 50, 1e-8)
        assert abs(infos[c]["iters"] - io["iters"]) <= 1, (c, infos[c], io)


@pytest.mark.parametrize("n,leaf,prec", [(8, 64, "fp64"), (5, 20, "fp64"), (4, 8, "fp32"), (8, 32, "fp32"),
                                          (16, 64, "fp64"), (8, 128, "fp64")])
def test_persistent_solve_matches_wave_solve(gpu, n, leaf, prec, monkeypatch):
    """The persistent left-looking H-solve equals the planned recursive
    H-solve (same arithmetic, different summation order).  With FP32
    factors the planned form also rounds its intermediate vectors to FP32
    (the persistent form keeps them in FP64), hence the looser bound."""
    import torch
    hlu, inputs = _lib()
    A, (rp, ci, va, mid) = _setup(n, 4.0, leaf)
    H = hlu.HLU(rp, ci, va, mid, 2.0, leaf).hlu_factor(1e-4, prec=prec)
    for nrhs in (1, 5, 33):
        b = torch.tensor(inputs.exact_solution_cols(A.n, nrhs, seed=7), device="cuda")
        monkeypatch.setenv("HLU_DEBUG_WAVE_SOLVE", "1")
        z_w = H.hlu_solve(b)
        monkeypatch.delenv("HLU_DEBUG_WAVE_SOLVE")
        tol = 1e-10 if prec == "fp64" else 1e-4
        for rep in range(3):   # the persistent form is scheduled dynamically: repeat
            z_p = H.hlu_solve(b)
            torch.cuda.synchronize()
            assert torch.isfinite(z_p).all()
            assert (z_p - z_w).norm() <= tol * z_w.norm(), (nrhs, rep, (z_p - z_w).norm().item(), z_w.norm().item())


def test_solve_timing_counts_launches(gpu):
    """hlu_set_timing brackets each persistent solve launch (at most 32
    columns each) with events; hlu_get_stats reports count, columns, time."""
    import torch
    hlu, inputs = _lib()
    A, (rp, ci, va, mid) = _setup(4, 2.0, 32)
    H = hlu.HLU(rp, ci, va, mid, 2.0, 32).hlu_factor(1e-6, prec="fp64")
    H.hlu_set_timing(True)
    for nrhs in (5, 33):
        H.hlu_solve(torch.tensor(inputs.exact_solution_cols(A.n, nrhs, seed=1), device="cuda"))
    st = H.hlu_get_stats()
    assert st["solve_launches"] == 3 and st["solve_columns"] == 38
    assert st["solve_kernel_ms"] > 0
    H.hlu_set_timing(False)
    H.hlu_solve(torch.tensor(inputs.exact_solution_cols(A.n, 2, seed=1), device="cuda"))
    st = H.hlu_get_stats()
    assert st["solve_launches"] == 0 and st["solve_columns"] == 0


def test_autotune_leaf(gpu):
    """The autotuner times every candidate (factor + GMRES on the device) and
    returns the fastest one."""
    hlu, _ = _lib()
    leaves = (8, 16, 32)
    best, secs = hlu.hlu_autotune_leaf(4, 2.0, leaves=leaves, eps=1e-6, prec="fp64", restart=30, tol=1e-10)
    assert all(np.isfinite(s) and s > 0 for s in secs), secs
    assert best == leaves[int(np.argmin(secs))]


@pytest.mark.parametrize("leaf", [96, 128])
def test_large_leaves_against_oracle(gpu, leaf):
    """Leaf sizes above the chain's 64 register rows (the autotuner's larger
    candidates): FP32 factor within the FP32 bound of the oracle's, GMRES
    iterations +-1."""
    import torch
    hlu, inputs = _lib()
    n, kappa, eps = 8, 4.0, 1e-3
    A, (rp, ci, va, mid) = _setup(n, kappa, leaf)
    H = hlu.HLU(rp, ci, va, mid, 2.0, leaf).hlu_factor(eps, prec="fp32")
    d, s = oracle_problem(n, kappa, leaf)
    o = oracle_factor(n, kappa, leaf, eps)
    e_gpu = gpu_factor_error(H, d.A, s.perm)
    bar = fp32_factor_bound(o.factor_error(), o.factor_error(storage=np.float32), leaf)
    assert e_gpu <= bar, (e_gpu, o.factor_error(), bar)
    X = inputs.exact_solution_cols(A.n, 3, seed=5)
    B = (d.A @ X.T).T.copy()
    x, infos = hlu.gmres_solve(A, torch.tensor(B, device="cuda"), H, restart=50, tol=1e-8)
    xg = x.cpu().numpy()
    for c in range(3):
        relres = np.linalg.norm(d.A @ xg[c] - B[c]) / np.linalg.norm(B[c])
        assert infos[c]["converged"] and relres <= 1e-8
        _, io = oracle_solve(n, kappa, leaf, eps, B[c], 50, 1e-8)
        assert abs(infos[c]["iters"] - io["iters"]) <= 1, (c, infos[c], io)


def test_caller_owned_solve_workspace(gpu):
    """hlu_bind_solve_workspace: the persistent solve's buffers in caller
    memory give the same results, bit for bit, as library-owned ones."""
    import torch
    hlu, inputs = _lib()
    A, (rp, ci, va, mid) = _setup(8, 4.0, 64)
    Ha = hlu.HLU(rp, ci, va, mid, 2.0, 64).hlu_factor(1e-4, prec="fp32")
    Hb = hlu.HLU(rp, ci, va, mid, 2.0, 64)
    nb = Hb.hlu_bind_solve_workspace(1e-4, prec="fp32")
    Hb.hlu_factor(1e-4, prec="fp32")
    assert nb > 0
    v = torch.tensor(inputs.exact_solution_cols(A.n, 5, seed=9), device="cuda")
    za, zb = Ha.hlu_solve(v), Hb.hlu_solve(v)
    torch.cuda.synchronize()
    assert torch.equal(za, zb)
    x, infos = hlu.gmres_solve(A, A.hlu_spmv(v), Hb, restart=30, tol=1e-10)
    assert all(i["converged"] for i in infos)


@pytest.mark.parametrize("boxes,beta", [(True, None), (False, 10.0)])
def test_support_boxes_and_coefficient_against_oracle(gpu, boxes, beta):
    """Admissibility on the basis functions' supports (hlu_build_boxes) and a
    piecewise constant curl-curl coefficient (hlu_kuhn_assemble_beta, a block
    of beta = 10 in the middle of the cube), each against the oracle built
    the same way: FP64 factor error within 2x the oracle's, GMRES iterations
    within +-1, final relative residual <= 1e-8."""
    import scipy.sparse as sp
    import torch
    from paper_2211_11303_amd import hlu, inputs
    from oracle.assemble import Discretisation
    from oracle.cluster import Structure
    from oracle.hmatrix import HLU as OracleHLU
    from oracle.krylov import gmres as oracle_gmres
    n, kappa, leaf, eps, box = 8, 4.0, 32, 1e-2, (2, 2, 2, 6, 6, 6)
    d = Discretisation(n, kappa, box if beta else None, beta or 1.0)
    s = Structure(d.mesh.midpoints2(), leaf, 2.0, boxes=d.mesh.support_boxes2() if boxes else None)
    o = OracleHLU(s, d.A, eps).factor()
    if beta:
        rp, ci, va, mid = hlu.hlu_kuhn_assemble_beta(n, kappa, box, beta)
    else:
        rp, ci, va, mid = hlu.hlu_kuhn_assemble(n, kappa)
    H = hlu.HLU(rp, ci, va, mid, 2.0, leaf, boxes=hlu.hlu_kuhn_support_boxes(n) if boxes else None)
    H.hlu_factor(eps, prec="fp64")
    st = H.hlu_export_structure()
    assert np.array_equal(st["bkind"], [b.kind for b in s.block_leaves])
    Acsr = sp.csr_matrix((va, ci, rp), shape=(d.N, d.N))
    e_or = o.factor_error()
    e_gpu = gpu_factor_error(H, Acsr, st["perm"])
    assert e_gpu <= 2 * e_or + 1e-12, (e_gpu, e_or)
    A = hlu.SpMat(rp, ci, va)
    X = inputs.exact_solution_cols(d.N, 4, seed=3)
    B = (d.A @ X.T).T.copy()
    x, infos = hlu.gmres_solve(A, torch.tensor(B, device="cuda"), H, restart=50, tol=1e-8)
    xg = x.cpu().numpy()
    for c in range(4):
        _, io = oracle_gmres(d.A, B[c], o.solve, restart=50, tol=1e-8, max_iters=2000)
        assert infos[c]["converged"] and abs(infos[c]["iters"] - io["iters"]) <= 1, (c, infos[c], io)
        assert np.linalg.norm(Acsr @ xg[c] - B[c]) <= 1e-8 * np.linalg.norm(B[c])


@pytest.mark.parametrize("prec", ["fp64", "fp32"])
def test_fitted_rank_capacity(gpu, prec):
    """hlu_fit_ranks: capacities fitted to the measured eps-ranks give the
    same factorisation (bit for bit: no truncation is cut) in a smaller
    workspace; fitting from a capped run (max_rank 8) converges to it in a
    few refits; GMRES against the oracle as for the uniform capacity."""
    import torch
    hlu, inputs = _lib()
    n, kappa, leaf, eps = 8, 4.0, 32, 1e-4
    A, (rp, ci, va, mid) = _setup(n, kappa, leaf)
    H = hlu.HLU(rp, ci, va, mid, 2.0, leaf).hlu_factor(eps, prec=prec)
    st0 = H.hlu_get_stats()
    ranks0 = H.hlu_get_ranks()
    V = torch.tensor(inputs.exact_solution_cols(A.n, 5, seed=4), device="cuda")
    y0 = H.hlu_apply_lu(V).clone()
    z0 = H.hlu_solve(V).clone()
    nb = H.hlu_fit_ranks(eps, margin=0, prec=prec)
    H.hlu_factor(eps, prec=prec)
    st1 = H.hlu_get_stats()
    assert nb == st1["workspace_bytes"] < st0["workspace_bytes"]
    assert st1["rank_capacity_entries"] < 0.6 * st0["rank_capacity_entries"], (st0, st1)
    assert st1["capped_blocks"] == 0
    assert np.array_equal(H.hlu_get_ranks(), ranks0)
    assert torch.equal(H.hlu_apply_lu(V), y0)
    assert torch.equal(H.hlu_solve(V), z0)
    # from a capped run: ranks cut at 8, then refit until nothing is cut
    G = hlu.HLU(rp, ci, va, mid, 2.0, leaf).hlu_factor(eps, max_rank=8, prec=prec)
    assert G.hlu_get_stats()["capped_blocks"] > 0
    for refit in range(4):
        G.hlu_fit_ranks(eps, margin=2, prec=prec)
        G.hlu_factor(eps, prec=prec, allow_overflow=True)
        if G.hlu_get_stats()["capped_blocks"] == 0:
            break
    assert G.hlu_get_stats()["capped_blocks"] == 0, refit
    assert np.array_equal(G.hlu_get_ranks(), ranks0)
    assert torch.equal(G.hlu_apply_lu(V), y0)
    # GMRES with the fitted factor against the oracle's iterations
    d, s = oracle_problem(n, kappa, leaf)
    B = (d.A @ inputs.exact_solution_cols(A.n, 2, seed=6).T).T.copy()
    x, infos = hlu.gmres_solve(A, torch.tensor(B, device="cuda"), G, restart=50, tol=1e-8)
    for c in range(2):
        _, io = oracle_solve(n, kappa, leaf, eps, B[c], 50, 1e-8)
        assert infos[c]["converged"] and abs(infos[c]["iters"] - io["iters"]) <= 1
    # back to the uniform capacity
    assert G.hlu_fit_ranks(eps, margin=-1, prec=prec) == st0["workspace_bytes"]


@pytest.mark.parametrize("prec", ["fp64", "fp32"])
def test_two_box_domain_against_oracle(gpu, prec):
    """The two-box domain of Example 2 on the lattice (m = 2 cubes per unit,
    n = 8, N = 1,406; kappa 8 in the unit-cube frame, i.e. 2 on the
    paper's 4-unit domain; eps 1e-2, 6-8 oracle iterations; source
    J = (1, 1, 1) as in Example 2, and random x*):
    factor error within the FP64 / FP32 bars of the oracle's, GMRES
    iterations within +-1, final relative residual <= 1e-8."""
    import scipy.sparse as sp
    import torch
    from paper_2211_11303_amd import hlu, inputs
    from oracle.assemble import Discretisation
    from oracle.cluster import Structure
    from oracle.hmatrix import HLU as OracleHLU
    from oracle.krylov import gmres as oracle_gmres
    n, mask = inputs.two_box_mask(2)
    kappa, leaf, eps = 8.0, 32, 1e-2
    d = Discretisation(n, kappa, mask=mask)
    s = Structure(d.mesh.midpoints2(), leaf, 2.0)
    o = OracleHLU(s, d.A, eps).factor()
    rp, ci, va, mid = hlu.hlu_kuhn_assemble_domain(n, kappa, mask)
    H = hlu.HLU(rp, ci, va, mid, 2.0, leaf).hlu_factor(eps, prec=prec)
    st = H.hlu_export_structure()
    assert np.array_equal(st["perm"], s.perm)
    Acsr = sp.csr_matrix((va, ci, rp), shape=(d.N, d.N))
    e_or = o.factor_error()
    bar = 2 * e_or + 1e-12 if prec == "fp64" else fp32_factor_bound(e_or, o.factor_error(storage=np.float32), leaf)
    e_gpu = gpu_factor_error(H, Acsr, st["perm"])
    assert e_gpu <= bar, (e_gpu, e_or, bar)
    A = hlu.SpMat(rp, ci, va)
    B = np.stack([d.load((1.0, 1.0, 1.0))] + list((d.A @ inputs.exact_solution_cols(d.N, 3, seed=5).T).T))
    x, infos = hlu.gmres_solve(A, torch.tensor(B, device="cuda"), H, restart=50, tol=1e-8)
    xg = x.cpu().numpy()
    for c in range(B.shape[0]):
        _, io = oracle_gmres(d.A, B[c], o.solve, restart=50, tol=1e-8, max_iters=2000)
        assert infos[c]["converged"] and abs(infos[c]["iters"] - io["iters"]) <= 1, (c, infos[c], io)
        assert np.linalg.norm(Acsr @ xg[c] - B[c]) <= 1e-8 * np.linalg.norm(B[c])


def test_gmres_refined_near_resonance(gpu):
    """gmres_solve_refined with kappa^2 0.1 % below a cavity eigenvalue (4^3,
    leaf 8): GMRES with the eps = 0.1 factor needs more than 20 iterations;
    with a first-try budget of 20 and eps_factor 0.01 the handle is refactored
    once (eps 1e-3) and both columns converge within 20, equal bit for bit to
    GMRES with a handle factored at 1e-3 directly; against the oracle's GMRES
    with its own H-LU at 1e-3: iterations within +-1."""
    import scipy.sparse as sp
    import torch
    from oracle.assemble import Discretisation
    from oracle.cluster import Structure
    from oracle.hmatrix import HLU as OracleHLU
    from oracle.krylov import gmres as oracle_gmres
    from test_gpu_serving import _near_resonant_kappa
    hlu, inputs = _lib()
    n, leaf = 4, 8
    kappa = _near_resonant_kappa(n, 1e-3)
    rp, ci, va, mid = hlu.hlu_kuhn_assemble(n, kappa)
    A = hlu.SpMat(rp, ci, va)
    Acsr = sp.csr_matrix((va, ci, rp), shape=(A.n, A.n))
    B = np.stack([Acsr @ x for x in inputs.exact_solution_cols(A.n, 2, seed=5)])
    Bt = torch.tensor(B, device="cuda")
    H = hlu.HLU(rp, ci, va, mid, 2.0, leaf).hlu_factor(0.1, prec="fp64")
    _, plain = hlu.gmres_solve(A, Bt, H, restart=30, tol=1e-10, max_iters=300)
    assert all(i["converged"] for i in plain) and min(i["iters"] for i in plain) > 20, plain
    x, infos, refines = hlu.gmres_solve_refined(A, Bt, H, restart=30, tol=1e-10, max_iters=300, refine_iters=20,
                                                max_refines=2, eps_factor=0.01)
    assert refines == 1
    assert all(i["converged"] and i["iters"] <= 20 for i in infos), infos
    H2 = hlu.HLU(rp, ci, va, mid, 2.0, leaf).hlu_factor(1e-3, prec="fp64")
    x2, i2 = hlu.gmres_solve(A, Bt, H2, restart=30, tol=1e-10, max_iters=300)
    assert torch.equal(x, x2) and [i["iters"] for i in infos] == [i["iters"] for i in i2]
    d = Discretisation(n, kappa)
    o = OracleHLU(Structure(d.mesh.midpoints2(), leaf, 2.0), d.A, 1e-3).factor()
    for c in range(2):
        _, io = oracle_gmres(d.A, B[c], o.solve, restart=30, tol=1e-10, max_iters=300)
        assert abs(infos[c]["iters"] - io["iters"]) <= 1, (c, infos[c], io)
    # nothing left to refine: a column that misses tol is reported
    with pytest.raises(Exception):
        hlu.gmres_solve_refined(A, Bt, H2, restart=30, tol=1e-10, max_iters=3, refine_iters=2, max_refines=0,
                                eps_factor=0.1)
