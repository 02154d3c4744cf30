"""Serving runtime (hlu_server_*): continuous batching, admission by device
bytes, cache eviction.

Each GMRES column keeps its own Krylov process and every kernel computes a
column with the same arithmetic whatever its companions, so a request's
result is expected to be the same alone and in a mix: the bar is equal
iteration counts and |x_mix - x_alone| <= 1e-14 |x_alone| per request."""
import numpy as np
import pytest

pytestmark = pytest.mark.gpu


def _csr(n, kappa):
    import scipy.sparse as sp
    from paper_2211_11303_amd import hlu
    rp, ci, va, _ = hlu.hlu_kuhn_assemble(n, kappa)
    return sp.csr_matrix((va, ci, rp), shape=(len(rp) - 1, len(rp) - 1))


def _request_set():
    from paper_2211_11303_amd import inputs
    reqs = []
    # repeated (n, kappa) pairs so that requests share factors and GMRES calls
    for i, (n, kappa, nrhs) in enumerate([(4, 2.0, 1), (5, 3.0, 2), (4, 2.0, 3), (6, 1.5, 1), (5, 3.0, 1),
                                          (4, 2.0, 2), (4, 7.0, 1), (6, 1.5, 4), (5, 3.0, 3), (4, 2.0, 1)]):
        N = inputs.num_interior_edges(n)
        xs = inputs.exact_solution_cols(N, nrhs, seed=100 + i)
        A = _csr(n, kappa)
        reqs.append(dict(n=n, kappa=kappa, xs=xs, b=np.stack([A @ x for x in xs]), A=A))
    return reqs


def test_result_same_alone_and_in_mix(gpu):
    from paper_2211_11303_amd import hlu
    reqs = _request_set()
    srv = hlu.Server(workers=3, max_batch_rhs=8, hbm_budget=8 << 30, leaf=32, eps=1e-6, prec="fp64",
                     restart=30, tol=1e-10)
    for n in (4, 5, 6):
        srv.hlu_server_prepare(n)
    tickets = [srv.hlu_server_submit(r["n"], r["kappa"], r["b"]) for r in reqs]
    mix = [srv.hlu_server_wait(t) for t in tickets]
    st = srv.hlu_server_get_stats()
    srv.close()
    assert st["completed"] == len(reqs) and st["failed"] == 0
    assert st["factorizations"] == 4          # distinct (n, kappa) pairs
    assert st["gmres_calls"] < len(reqs)      # some requests shared a call
    for r, (x, infos, q, lat) in zip(reqs, mix):
        for c in range(len(x)):
            assert infos[c]["converged"]
            assert np.linalg.norm(r["A"] @ x[c] - r["b"][c]) <= 1e-10 * np.linalg.norm(r["b"][c])
        assert lat >= q >= 0
    # each request alone, on a fresh server
    for r, (x, infos, _, _) in zip(reqs, mix):
        one = hlu.Server(workers=1, max_batch_rhs=8, hbm_budget=8 << 30, leaf=32, eps=1e-6, prec="fp64",
                         restart=30, tol=1e-10)
        xa, ia, _, _ = one.hlu_server_wait(one.hlu_server_submit(r["n"], r["kappa"], r["b"]))
        one.close()
        assert [i["iters"] for i in ia] == [i["iters"] for i in infos]
        assert np.abs(xa - x).max() <= 1e-14 * np.abs(xa).max()


def test_admission_evicts_and_rejects(gpu):
    from paper_2211_11303_amd import hlu, inputs
    from paper_2211_11303_amd import _lib as L
    # footprint of one 6^3 factor, to size a budget that holds just one
    rp, ci, va, mid = hlu.hlu_kuhn_assemble(6, 1.0)
    import ctypes
    H = hlu.HLU(rp, ci, va, mid, 2.0, 32)
    o = L.FactorOpts(1e-6, 32, L.HLU_FP64)
    nb, npl = ctypes.c_size_t(), ctypes.c_size_t()
    L.check(L.lib().hlu_device_bytes(H.handle, ctypes.byref(o), ctypes.byref(nb)))
    L.check(L.lib().hlu_plan_device_bytes(H.handle, ctypes.byref(o), ctypes.byref(npl)))
    assert 0 < npl.value < nb.value
    # the mesh's shared plans once, and room for 1.6 factors
    budget = int(npl.value + (nb.value - npl.value) * 1.6)
    srv = hlu.Server(workers=2, max_batch_rhs=4, hbm_budget=budget, leaf=32, eps=1e-6, max_rank=32,
                     prec="fp64", restart=30, tol=1e-10)
    N = inputs.num_interior_edges(6)
    tickets = []
    for i, kappa in enumerate([1.0, 2.0, 3.0, 1.0]):
        b = _csr(6, kappa) @ inputs.exact_solution_cols(N, 1, seed=i)[0]
        tickets.append(srv.hlu_server_submit(6, kappa, b))
    for t in tickets:
        x, infos, _, _ = srv.hlu_server_wait(t)
        assert infos[0]["converged"]
    st = srv.hlu_server_get_stats()
    assert st["peak_bytes"] <= budget
    assert st["evictions"] >= 2 and st["factorizations"] >= 3
    # a mesh whose factor can never fit the budget is refused, not queued forever
    big = inputs.num_interior_edges(12)
    t = srv.hlu_server_submit(12, 1.0, np.ones(big))
    with pytest.raises(L.HluError) as e:
        srv.hlu_server_wait(t)
    assert e.value.status == L.STATUS_CODES["HLU_ERR_OUT_OF_MEMORY"]
    srv.close()


def _near_resonant_kappa(n, rel_gap):
    """kappa with kappa^2 just below the fourth non-zero eigenvalue of the
    discrete cavity problem K u = lambda M u (dense, small n)."""
    import scipy.linalg as sl
    from paper_2211_11303_amd import hlu
    K = _csr(n, 0.0).toarray()
    M = K - _csr(n, 1.0).toarray()
    w = sl.eigh(K, M, eigvals_only=True)
    w = w[w > 1e-6 * w.max()]
    return float(np.sqrt(w[3] * (1.0 - rel_gap)))


def test_refinement_near_resonance(gpu):
    """kappa^2 0.1% below a cavity eigenvalue: with eps = 0.1 (leaf 8) GMRES
    needs about 50 iterations, more than the first-try budget of 20, so the
    server refactors at eps = 1e-3 and the request converges in about 10.  A
    later request for the same (n, kappa) is served by the refined factor."""
    from paper_2211_11303_amd import inputs
    from paper_2211_11303_amd import hlu
    n = 4
    kappa = _near_resonant_kappa(n, 1e-3)
    A = _csr(n, kappa)
    N = inputs.num_interior_edges(n)
    b = np.stack([A @ x for x in inputs.exact_solution_cols(N, 2, seed=5)])
    common = dict(workers=1, max_batch_rhs=8, hbm_budget=4 << 30, leaf=8, eps=0.1, prec="fp64", restart=30,
                  max_iters=300, tol=1e-10)
    plain = hlu.Server(**common)
    xp, ip, _, _ = plain.hlu_server_wait(plain.hlu_server_submit(n, kappa, b))
    plain.close()
    assert all(i["converged"] for i in ip) and min(i["iters"] for i in ip) > 20, ip
    srv = hlu.Server(refine_iters=20, max_refines=2, refine_eps_factor=0.01, **common)
    x, infos, _, _ = srv.hlu_server_wait(srv.hlu_server_submit(n, kappa, b))
    st = srv.hlu_server_get_stats()
    assert st["refinements"] == 1 and st["factorizations"] == 1, st
    for c in range(2):
        assert infos[c]["converged"] and infos[c]["iters"] <= 20, infos
        assert np.linalg.norm(A @ x[c] - b[c]) <= 1e-10 * np.linalg.norm(b[c])
    x2, i2, _, _ = srv.hlu_server_wait(srv.hlu_server_submit(n, kappa, b[:1]))
    st = srv.hlu_server_get_stats()
    srv.close()
    assert st["refinements"] == 1 and st["cache_hits"] == 1, st
    assert i2[0]["iters"] == infos[0]["iters"]
    assert np.abs(x2[0] - x[0]).max() <= 1e-14 * np.abs(x[0]).max()


@pytest.mark.parametrize("prec,eps", [("fp64", 1e-6), ("fp32", 1e-4)])
def test_requests_against_oracle(gpu, prec, eps):
    """Every request answered by a mixed serving run against the oracle's
    GMRES on the same right-hand sides with the oracle's H-LU at the same
    eps and leaf: iterations within +-1 per column, true relative residual
    <= tol, and ||x - x_oracle|| <= 3 max(e_or, a res) relative (e_or the
    oracle's error against x*, a = e_or / its final residual, res the
    server's final residual; both solve to the same residual tolerance)."""
    from gpu_util import oracle_solve
    from paper_2211_11303_amd import hlu
    reqs = _request_set()
    leaf = 32
    srv = hlu.Server(workers=3, max_batch_rhs=8, hbm_budget=8 << 30, leaf=leaf, eps=eps, prec=prec,
                     restart=30, tol=1e-10)
    tickets = [srv.hlu_server_submit(r["n"], r["kappa"], r["b"]) for r in reqs]
    out = [srv.hlu_server_wait(t) for t in tickets]
    srv.close()
    for i, (r, (x, infos, _, _)) in enumerate(zip(reqs, out)):
        for c in range(len(x)):
            xo, io = oracle_solve(r["n"], r["kappa"], leaf, eps, r["b"][c], 30, 1e-10)
            rel = np.linalg.norm(r["A"] @ x[c] - r["b"][c]) / np.linalg.norm(r["b"][c])
            err_or = np.linalg.norm(xo - r["xs"][c]) / np.linalg.norm(r["xs"][c])
            d_or = np.linalg.norm(x[c] - xo) / np.linalg.norm(xo)
            assert infos[c]["converged"] and rel <= 1e-10, (i, c, infos[c], rel)
            assert abs(infos[c]["iters"] - io["iters"]) <= 1, (i, c, infos[c], io)
            rel_or = np.linalg.norm(r["A"] @ xo - r["b"][c]) / np.linalg.norm(r["b"][c])
            amp = err_or / max(rel_or, 1e-300)   # residual amplification (see test_gpu_cfg2)
            assert d_or <= 3 * max(err_or, amp * rel, 1e-14), (i, c, d_or, err_or)
