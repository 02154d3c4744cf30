"""H-matrix inverse by the Schulz iteration and its use as a preconditioner.

Test infrastructure (see the package header).  Plain FP64 code.

Sec. 3 obtains an approximate inverse B_H of the H-matrix A_H with the
iterative method of Schulz, and Sec. 4 computes it with truncated SVDs of
rank r in the admissible blocks (Example 2 uses B_H as the preconditioner).
The Schulz iteration for the inverse is

    X_{k+1} = X_k (2 I - A X_k),

whose residual R_k = I - A X_k satisfies R_{k+1} = R_k^2: it converges
quadratically once ||R_k|| < 1.  Here both products are formed in
H-arithmetic on the block tree of A, with the same H-products and the same
truncation after every addition into a low-rank block as the H-LU:

    Z = 2 I - A X_k,      X_{k+1} = X_k Z.

Start: X_0 = A^T / (||A||_1 ||A||_inf).  Then X_0 A = A^T A / (||A||_1
||A||_inf) is symmetric with eigenvalues in (0, 1] (||A||_2^2 <=
||A||_1 ||A||_inf), so R_0 has spectral radius below 1 for every
nonsingular A and the iteration converges.

The iteration stops when the probed residual
rho_k = ||(I - A X_k) Omega||_F / ||Omega||_F (Omega: N x 8 standard normal
from numpy's default_rng(12345), cluster order) is at most tol, when it did
not decrease in the last step (the truncation floor; the previous iterate
is kept), or after max_iters steps.
"""

import numpy as np
import scipy.sparse as sp

from .cluster import DENSE, LOWRANK
from .hmatrix import HMatrix, Truncation, gemm, hmul


def _add_identity(H, alpha):
    """H += alpha I: the diagonal leaves are dense."""
    for b in H.root.leaves():
        if b.r0 == b.c0 and b.r1 == b.c1:
            assert b.kind == DENSE
            b.D = b.D + alpha * np.eye(b.m)


def _negate(H):
    for b in H.root.leaves():
        if b.kind == DENSE:
            b.D = -b.D
        elif b.kind == LOWRANK:
            b.X = -b.X


class HInverse:
    """B_H ~ A^{-1} by the Schulz iteration in H-arithmetic."""

    def __init__(self, structure, A_csr, eps, max_rank=0):
        self.structure = structure
        self.trunc = Truncation(eps, max_rank)
        self.A = A_csr.tocsr()
        self.perm = structure.perm
        self.Ap = self.A[self.perm][:, self.perm].tocsr()
        self.H_A = HMatrix(structure, self.A, self.trunc)   # A_H (Algorithm 1, step I)
        a = abs(self.A)
        self.alpha = 1.0 / (a.sum(axis=0).max() * a.sum(axis=1).max())
        self.X = HMatrix(structure, (self.A.T * self.alpha).tocsr(), self.trunc)
        self.history = []
        self._zero = sp.csr_matrix(self.A.shape)
        self._probe = np.random.default_rng(12345).standard_normal((structure.N, 8))

    def residual(self, X=None):
        """rho = ||(I - A X) Omega||_F / ||Omega||_F, cluster order."""
        X = X or self.X
        Om = self._probe
        return float(np.linalg.norm(Om - self.Ap @ hmul(X.root, Om)) / np.linalg.norm(Om))

    def step(self, X):
        """One Schulz step in H-arithmetic: Z = 2I - A X, return X Z."""
        Z = HMatrix(self.structure, self._zero, self.trunc)
        gemm(Z.root, self.H_A.root, X.root, self.trunc)      # Z = -A X
        _add_identity(Z, 2.0)                                # Z = 2I - A X
        W = HMatrix(self.structure, self._zero, self.trunc)
        gemm(W.root, X.root, Z.root, self.trunc)             # W = -X Z
        _negate(W)
        return W

    def compute(self, tol=1e-10, max_iters=100):
        rho = self.residual()
        self.history = [rho]
        for _ in range(max_iters):
            if rho <= tol:
                break
            Xn = self.step(self.X)
            rn = self.residual(Xn)
            if rn >= rho:
                break
            self.X, rho = Xn, rn
            self.history.append(rho)
        return self

    @property
    def iterations(self):
        return len(self.history) - 1

    def solve(self, r):
        """z = P^T B_H P r (natural order)."""
        r = np.asarray(r, dtype=np.float64)
        vec = r.ndim == 1
        R = r.reshape(len(r), -1)
        z = hmul(self.X.root, R[self.perm])
        out = np.empty_like(z)
        out[self.perm] = z
        return out[:, 0] if vec else out
