"""Pins for the oracle's truncated arithmetic, H-LU and H-solves
(Algorithm 1, steps II-III; truncated SVD of Sec. 4)."""
import numpy as np
import pytest

from oracle import hmatrix
from oracle.assemble import Discretisation
from oracle.cluster import Structure
from oracle.hmatrix import HLU, Truncation


def _problem(n, leaf, kappa):
    d = Discretisation(n, kappa)
    s = Structure(d.mesh.midpoints2(), leaf, 2.0)
    return d, s


def _dense_lu_nopiv(A):
    """Textbook unpivoted Doolittle LU, written out independently."""
    A = np.array(A, dtype=float)
    n = len(A)
    L = np.eye(n)
    U = np.zeros_like(A)
    for i in range(n):
        U[i, i:] = A[i, i:] - L[i, :i] @ U[:i, i:]
        L[i + 1:, i] = (A[i + 1:, i] - L[i + 1:, :i] @ U[:i, i]) / U[i, i]
    return L, U


def test_truncation_is_best_approximation():
    """Eckart-Young: the truncated sum is the best rank-k approximation of
    X Y^T, with spectral error sigma_{k+1}."""
    rng = np.random.default_rng(3)
    X = rng.standard_normal((40, 12)) @ np.diag(2.0 ** -np.arange(12))
    Y = rng.standard_normal((30, 12))
    P = X @ Y.T
    s = np.linalg.svd(P, compute_uv=False)
    for eps in (1e-1, 1e-2, 1e-3):
        Xt, Yt = Truncation(eps)(X, Y)
        k = Xt.shape[1]
        assert k == int(np.sum(s > eps * s[0]))
        assert abs(np.linalg.norm(P - Xt @ Yt.T, 2) - s[k]) <= 1e-12 * s[0]
    Xt, Yt = Truncation(1e-12, max_rank=3)(X, Y)
    assert Xt.shape[1] == 3
    assert abs(np.linalg.norm(P - Xt @ Yt.T, 2) - s[3]) <= 1e-12 * s[0]
    Xt, Yt = Truncation(0.0)(X, np.zeros_like(Y))
    assert Xt.shape[1] == 0


def test_truncation_fallback_driver_is_best_approximation(monkeypatch):
    """The truncation's second SVD driver (taken when the first reports no
    convergence) obeys the same Eckart-Young pin.  The first driver is made
    to fail here; the reference singular values are computed beforehand."""
    rng = np.random.default_rng(5)
    X = rng.standard_normal((36, 10)) @ np.diag(3.0 ** -np.arange(10))
    Y = rng.standard_normal((28, 10))
    P = X @ Y.T
    s = np.linalg.svd(P, compute_uv=False)

    failed = []

    def no_convergence(*args, **kwargs):
        failed.append(1)
        raise np.linalg.LinAlgError("SVD did not converge")

    monkeypatch.setattr(hmatrix.np.linalg, "svd", no_convergence)
    for eps in (1e-1, 1e-3):
        Xt, Yt = Truncation(eps)(X, Y)
        k = Xt.shape[1]
        assert k == int(np.sum(s > eps * s[0]))
        E = P - Xt @ Yt.T
        monkeypatch.undo()   # the check's own spectral norm uses the first driver
        assert abs(np.linalg.norm(E, 2) - s[k]) <= 1e-12 * s[0]
        monkeypatch.setattr(hmatrix.np.linalg, "svd", no_convergence)
    assert len(failed) == 2


@pytest.mark.parametrize("n,leaf", [(4, 32), (4, 8), (5, 20), (3, 4)])
def test_untruncated_hlu_is_dense_lu(n, leaf):
    """eps = 0: the H-LU equals the unpivoted LU of P A P^T."""
    d, s = _problem(n, leaf, 2.0)
    Ap = d.A[s.perm][:, s.perm].toarray()
    h = HLU(s, d.A, 0.0).factor()
    F = h.H.to_dense()
    L, U = _dense_lu_nopiv(Ap)
    scale = np.abs(U).max()
    assert np.abs(np.tril(F, -1) - np.tril(L, -1)).max() <= 1e-10 * max(1, np.abs(L).max())
    assert np.abs(np.triu(F) - U).max() <= 1e-10 * scale
    # backward error of the factors
    LU = (np.tril(F, -1) + np.eye(len(F))) @ np.triu(F)
    assert np.linalg.norm(LU - Ap) / np.linalg.norm(Ap) <= 1e-12
    assert h.factor_error() <= 1e-12


def test_every_gemm_case_is_exercised():
    """The exactness check above runs every case of the H-product recursion."""
    hmatrix.GEMM_CASES.clear()
    for n, leaf in [(4, 32), (4, 8), (5, 20)]:
        d, s = _problem(n, leaf, 2.0)
        HLU(s, d.A, 0.0).factor()
    assert set(hmatrix.GEMM_CASES) == {
        "lowrank*any", "any*lowrank", "dense*dense->dense", "dense*dense->other",
        "dense*sub->dense", "dense*sub->other", "sub*dense->dense", "sub*dense->other",
        "sub*sub->sub", "sub*sub->lowrank"}


def test_hmatrix_products_against_dense():
    """hmul / hmulT against the dense matrix of an H-matrix with ranks."""
    d, s = _problem(4, 8, 2.0)
    h = HLU(s, d.A, 1e-3).factor()
    F = h.H.to_dense()
    V = np.random.default_rng(0).standard_normal((d.N, 3))
    assert np.allclose(hmatrix.hmul(h.H.root, V), F @ V, rtol=0, atol=1e-11 * np.abs(F).max())
    assert np.allclose(hmatrix.hmulT(h.H.root, V), F.T @ V, rtol=0, atol=1e-11 * np.abs(F).max())


@pytest.mark.parametrize("eps", [1e-2, 1e-4, 1e-6])
def test_solve_inverts_factors(eps):
    """U^{-1} L^{-1} (L U y) = y for any truncation."""
    d, s = _problem(4, 8, 2.0)
    h = HLU(s, d.A, eps).factor()
    y = np.random.default_rng(1).standard_normal((d.N, 2))
    F = h.H.to_dense()
    L = np.tril(F, -1) + np.eye(d.N)
    U = np.triu(F)
    assert np.allclose(h.apply_LU(y), L @ (U @ y), atol=1e-12 * np.abs(L @ U).max())
    r = np.empty_like(y)
    r[s.perm] = L @ (U @ y)                 # natural order
    z = h.solve(r)
    assert np.linalg.norm(z[s.perm] - y) <= 1e-10 * np.linalg.norm(y)


def test_factor_error_follows_eps():
    """The factor error decreases with eps and stays below eps."""
    d, s = _problem(6, 16, 4.0)
    errs = []
    for eps in (1e-2, 1e-4, 1e-6, 1e-8):
        h = HLU(s, d.A, eps).factor()
        errs.append(h.factor_error())
        assert errs[-1] <= eps
    assert all(a > b for a, b in zip(errs, errs[1:]))


def test_zero_pivot_detected():
    D = np.array([[0.0, 1.0], [1.0, 0.0]])
    with pytest.raises(hmatrix.ZeroPivot):
        hmatrix.getrf_nopiv(D)


@pytest.mark.parametrize("n,leaf,rtol", [(4, 32, 1e-3), (4, 8, 0.5)])
def test_fp32_storage_error_matches_dense(n, leaf, rtol):
    """factor_error(storage=float32) of the untruncated H-LU against the same
    probe error of the textbook dense LU of P A P^T with L and U rounded to
    FP32 (the exact factors are the dense LU, so only the rounding differs):
    equal where the factors are stored densely (leaf 32 at 4^3); where many
    blocks are stored as X Y^T (leaf 8), X and Y are rounded instead of
    their product, the same order of error.  storage=float64 leaves the
    error unchanged."""
    d, s = _problem(n, leaf, 2.0)
    h = HLU(s, d.A, 0.0).factor()
    Ap = d.A.toarray()[np.ix_(s.perm, s.perm)]
    L, U = _dense_lu_nopiv(Ap)
    Om = np.random.default_rng(12345).standard_normal((len(Ap), 8))
    L32 = L.astype(np.float32).astype(float)
    U32 = U.astype(np.float32).astype(float)
    ref = Ap @ Om
    e_dense32 = np.linalg.norm(L32 @ (U32 @ Om) - ref) / np.linalg.norm(ref)
    e32 = h.factor_error(storage=np.float32)
    assert abs(e32 - e_dense32) <= rtol * e_dense32, (e32, e_dense32)
    assert 1e-9 < e32 < 1e-5
    assert h.factor_error() == h.factor_error(storage=np.float64) < 1e-12
