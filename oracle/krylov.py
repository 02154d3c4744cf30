"""Preconditioned Krylov solvers.

Test infrastructure (see the package header).

Sec. 4 (Example 1) solves the Galerkin system with GMRES preconditioned by
the H-LU factors, restarted after a fixed number of iterations and stopped
on the relative residual.  The paper does not fix the variant; here:

* right preconditioning, flexible storage (Z_j = M^{-1} v_j kept), x0 = 0;
* modified Gram-Schmidt Arnoldi, Givens rotations on the Hessenberg matrix;
* a cycle ends when the rotated residual |g_{j+1}| <= tol * ||b|| or after
  ``restart`` steps; then x += Z y and the true residual is formed;
* converged iff ||b - A x||_2 <= tol * ||b||_2, otherwise a new cycle starts;
* the iteration count is the number of Arnoldi steps (= preconditioner
  applications).

Algorithm 1, step III is the preconditioned Richardson iteration
x <- x + U^{-1}(L^{-1}(b - A x)), with the relative residual measured before
the correction and the loop left after it; step IV reports ||A x - b||_2.
"""

import numpy as np


def gmres(A, b, precond=None, restart=50, tol=1e-8, max_iters=1000):
    """Return (x, info) with info = dict(iters, converged, relres, abs_res)."""
    b = np.asarray(b, dtype=np.float64)
    N = len(b)
    M = precond if precond is not None else (lambda v: v)
    x = np.zeros(N)
    bnorm = np.linalg.norm(b)
    if bnorm == 0.0:
        return x, dict(iters=0, converged=True, relres=0.0, abs_res=0.0)
    iters = 0
    r = b.copy()
    while True:
        beta = np.linalg.norm(r)
        if beta <= tol * bnorm:
            return x, dict(iters=iters, converged=True, relres=beta / bnorm, abs_res=beta)
        if iters >= max_iters:
            return x, dict(iters=iters, converged=False, relres=beta / bnorm, abs_res=beta)
        m = restart
        V = np.zeros((N, m + 1))
        Z = np.zeros((N, m))
        H = np.zeros((m + 1, m))
        cs = np.zeros(m)
        sn = np.zeros(m)
        g = np.zeros(m + 1)
        g[0] = beta
        V[:, 0] = r / beta
        j_end = 0
        for j in range(m):
            Z[:, j] = M(V[:, j])
            w = A @ Z[:, j]
            for i in range(j + 1):                      # modified Gram-Schmidt
                H[i, j] = w @ V[:, i]
                w = w - H[i, j] * V[:, i]
            H[j + 1, j] = np.linalg.norm(w)
            if H[j + 1, j] != 0.0:
                V[:, j + 1] = w / H[j + 1, j]
            for i in range(j):                          # previous rotations
                t = cs[i] * H[i, j] + sn[i] * H[i + 1, j]
                H[i + 1, j] = -sn[i] * H[i, j] + cs[i] * H[i + 1, j]
                H[i, j] = t
            den = np.hypot(H[j, j], H[j + 1, j])
            cs[j], sn[j] = H[j, j] / den, H[j + 1, j] / den
            H[j, j] = den
            H[j + 1, j] = 0.0
            g[j + 1] = -sn[j] * g[j]
            g[j] = cs[j] * g[j]
            iters += 1
            j_end = j + 1
            if abs(g[j + 1]) <= tol * bnorm or iters >= max_iters or H[j, j] == 0.0:
                break
        y = np.zeros(j_end)
        for i in range(j_end - 1, -1, -1):              # back substitution
            y[i] = (g[i] - H[i, i + 1:j_end] @ y[i + 1:]) / H[i, i]
        x = x + Z[:, :j_end] @ y
        r = b - A @ x


def richardson(A, b, precond, tol=1e-8, max_iters=100):
    """Algorithm 1, steps III-IV; returns (x, info)."""
    b = np.asarray(b, dtype=np.float64)
    x = np.zeros(len(b))
    bnorm = np.linalg.norm(b)
    it = 0
    for it in range(1, max_iters + 1):
        r = b - A @ x
        err = np.linalg.norm(r) / bnorm
        x = x + precond(r)
        if err < tol:
            break
    error = np.linalg.norm(A @ x - b)
    return x, dict(iters=it, error=error, relres=error / bnorm)
