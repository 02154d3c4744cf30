"""Pins of the oracle's Schulz H-inverse (oracle/hinverse.py) against what
the mathematics fixes, independent of the oracle's own H-arithmetic:

* untruncated (eps = 0), every H-arithmetic iterate equals the dense Schulz
  iterate X_{k+1} = X_k (2I - A X_k) from the same start, formed with
  plain matrix products, and the dense iteration reaches inv(A);
* the residual identity R_{k+1} = R_k^2 (R_k = I - A X_k), checked on probe
  vectors through the H-iterates;
* the start X_0 = A^T / (||A||_1 ||A||_inf) gives eigenvalues of X_0 A in
  (0, 1] (the convergence condition);
* truncation: the final residual does not grow as eps decreases;
* the converged untruncated inverse is an exact preconditioner: GMRES
  stops after one iteration."""
import numpy as np
import pytest

from oracle.assemble import Discretisation
from oracle.cluster import Structure
from oracle.hinverse import HInverse
from oracle.hmatrix import hmul
from oracle.krylov import gmres


def _problem(n, kappa, leaf):
    d = Discretisation(n, kappa)
    return d, Structure(d.mesh.midpoints2(), leaf, 2.0)


def test_start_satisfies_convergence_condition():
    d, s = _problem(3, 2.0, 8)
    h = HInverse(s, d.A, 0.0)
    A = d.A.toarray()
    ev = np.linalg.eigvals(h.alpha * A.T @ A)
    assert np.all(ev.real > 0) and ev.real.max() <= 1.0 + 1e-12 and np.abs(ev.imag).max() < 1e-12


def test_untruncated_iterates_equal_dense_schulz():
    d, s = _problem(3, 2.0, 8)
    h = HInverse(s, d.A, 0.0)
    Ap = d.A.toarray()[np.ix_(s.perm, s.perm)]
    Xd = h.alpha * Ap.T
    X = h.X
    assert np.abs(X.to_dense() - Xd).max() <= 1e-14 * np.abs(Xd).max()
    I = np.eye(d.N)
    for k in range(8):
        X = h.step(X)
        Xd = Xd @ (2 * I - Ap @ Xd)
        err = np.abs(X.to_dense() - Xd).max() / np.abs(Xd).max()
        assert err <= 1e-10, (k, err)
    # the dense iteration itself converges to the inverse
    for _ in range(40):
        Xd = Xd @ (2 * I - Ap @ Xd)
    assert np.abs(Xd - np.linalg.inv(Ap)).max() <= 1e-9 * np.abs(np.linalg.inv(Ap)).max()


def test_residual_squares_each_step():
    d, s = _problem(3, 2.0, 8)
    h = HInverse(s, d.A, 0.0)
    Ap = h.Ap
    Om = np.random.default_rng(5).standard_normal((d.N, 3))

    def R(X, V):
        return V - Ap @ hmul(X.root, V)

    X = h.X
    for _ in range(5):
        Xn = h.step(X)
        lhs = R(Xn, Om)
        rhs = R(X, R(X, Om))
        assert np.linalg.norm(lhs - rhs) <= 1e-11 * max(np.linalg.norm(Om), 1.0)
        X = Xn


def test_truncation_trend():
    d, s = _problem(3, 2.0, 8)
    res = []
    for eps in (1e-1, 1e-2, 1e-3):
        h = HInverse(s, d.A, eps).compute(tol=1e-12, max_iters=60)
        res.append(h.history[-1])
    assert res[0] >= res[1] >= res[2], res
    assert res[2] < 1e-2


def test_converged_inverse_is_exact_preconditioner():
    d, s = _problem(3, 2.0, 8)
    h = HInverse(s, d.A, 0.0).compute(tol=1e-13, max_iters=80)
    assert h.history[-1] <= 1e-12
    b = d.A @ np.random.default_rng(1).uniform(-1, 1, d.N)
    x, info = gmres(d.A, b, h.solve, restart=30, tol=1e-10)
    assert info["converged"] and info["iters"] == 1
