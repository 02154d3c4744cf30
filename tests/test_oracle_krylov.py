"""Pins for the oracle's GMRES and Richardson iterations (Sec. 4,
Algorithm 1 steps III-IV)."""
import numpy as np
import pytest
import scipy.sparse as sp

from oracle.assemble import Discretisation
from oracle.cluster import Structure
from oracle.hmatrix import HLU
from oracle.krylov import gmres, richardson


def test_gmres_minimal_polynomial():
    """Without restart GMRES on a diagonalisable matrix with k distinct
    eigenvalues terminates in at most k steps (textbook property)."""
    rng = np.random.default_rng(5)
    Q, _ = np.linalg.qr(rng.standard_normal((40, 40)))
    lam = np.repeat([1.0, -2.0, 3.5, 7.0, -0.5], 8)
    A = Q @ np.diag(lam) @ Q.T
    b = rng.standard_normal(40)
    x, info = gmres(A, b, restart=40, tol=1e-12)
    assert info["converged"] and info["iters"] == 5
    assert np.allclose(A @ x, b, atol=1e-10)


def test_gmres_unpreconditioned_matches_dense_solve():
    d = Discretisation(3, 2.0)
    xs = np.random.default_rng(0).uniform(-1, 1, d.N)
    b = d.A @ xs
    x, info = gmres(d.A, b, restart=30, tol=1e-12, max_iters=5000)
    assert info["converged"]
    xd = np.linalg.solve(d.A.toarray(), b)
    assert np.linalg.norm(x - xd) <= 1e-8 * np.linalg.norm(xd)
    assert np.linalg.norm(b - d.A @ x) <= 1e-12 * np.linalg.norm(b)


def test_exact_preconditioner_one_iteration():
    d = Discretisation(4, 2.0)
    s = Structure(d.mesh.midpoints2(), 32, 2.0)
    h = HLU(s, d.A, 0.0).factor()
    b = d.A @ np.random.default_rng(1).uniform(-1, 1, d.N)
    x, info = gmres(d.A, b, h.solve, restart=30, tol=1e-10)
    assert info["iters"] == 1 and info["converged"]


def test_restart_and_stopping_rule():
    """A restarted run stops on the true residual and reports it."""
    rng = np.random.default_rng(2)
    A = sp.diags(np.linspace(1.0, 50.0, 200)).tocsr()
    b = rng.standard_normal(200)
    x, info = gmres(A, b, restart=5, tol=1e-9, max_iters=2000)
    assert info["converged"]
    assert info["relres"] <= 1e-9
    assert abs(info["relres"] - np.linalg.norm(b - A @ x) / np.linalg.norm(b)) < 1e-15
    x, info = gmres(A, b, restart=5, tol=1e-30, max_iters=7)
    assert not info["converged"] and info["iters"] == 7


def test_richardson_exact_preconditioner():
    """With the exact LU the Richardson loop of Algorithm 1 takes one
    correction; the error is measured before it, so the loop runs twice."""
    d = Discretisation(4, 2.0)
    s = Structure(d.mesh.midpoints2(), 32, 2.0)
    h = HLU(s, d.A, 0.0).factor()
    b = d.A @ np.random.default_rng(1).uniform(-1, 1, d.N)
    x, info = richardson(d.A, b, h.solve, tol=1e-8)
    assert info["iters"] == 2 and info["relres"] < 1e-12
