"""H-matrix storage, truncated arithmetic, H-LU factorisation and H-solves.

Test infrastructure (see the package header).  Plain recursive FP64 code.

Definition 1 (Sec. 3): on every admissible block (tau, sigma) the H-matrix is
a product X Y^T of rank r; the other leaves of the partition ("small blocks")
are stored densely.  Sec. 4 truncates low-rank blocks with the SVD,
U_r S_r V_r^T, keeping the leading r singular triplets.  Here the rank is
chosen per block from a relative threshold: keep sigma_i > eps * sigma_1
(eps = 0 keeps every non-zero triplet, i.e. no truncation), optionally capped
at ``max_rank`` (the paper's fixed-rank mode).

Algorithm 1, step II computes L and U blockwise in H-arithmetic.  The block
recursion used here is the standard one for a 2 x 2 partition
    L11 U11 = A11,   L11 U12 = A12,   L21 U11 = A21,
    L22 U22 = A22 - L21 U12,
applied on the block cluster tree down to the dense diagonal leaves, where an
unpivoted LU (L unit lower triangular) is taken.  In exact arithmetic it
equals the unpivoted LU of the permuted matrix.  Every product that lands in
a low-rank leaf is added with immediate truncation (QR of both factor stacks,
SVD of the small core).  Algorithm 1, step III applies the factors as
U^{-1}(L^{-1} r) by H-forward and H-backward substitution.

All index ranges are in cluster order (the permutation of the cluster tree).
"""

import numpy as np
import scipy.linalg as sla

from .cluster import DENSE, LOWRANK, SUB


class ZeroPivot(ArithmeticError):
    pass


# How often each case of ``gemm`` ran; the tests use it to show that every
# case of the recursion is exercised by the exactness checks.
GEMM_CASES = {}


def _case(name):
    GEMM_CASES[name] = GEMM_CASES.get(name, 0) + 1


class HBlock:
    """One node of the block tree with its storage."""

    __slots__ = ("r0", "r1", "c0", "c1", "kind", "D", "X", "Y", "sons", "row", "col")

    def __init__(self, node):
        self.row, self.col = node.row, node.col
        self.r0, self.r1 = node.row.begin, node.row.end
        self.c0, self.c1 = node.col.begin, node.col.end
        self.kind = node.kind
        self.D = self.X = self.Y = None
        self.sons = None
        if node.kind == SUB:
            self.sons = [[HBlock(node.sons[i][j]) for j in range(2)] for i in range(2)]

    @property
    def m(self):
        return self.r1 - self.r0

    @property
    def n(self):
        return self.c1 - self.c0

    def leaves(self):
        if self.kind == SUB:
            for row in self.sons:
                for s in row:
                    yield from s.leaves()
        else:
            yield self


class Truncation:
    """Rank rule for every low-rank addition: keep sigma_i > eps * sigma_1,
    at most ``max_rank`` triplets (0 = no cap)."""

    def __init__(self, eps, max_rank=0):
        self.eps = float(eps)
        self.max_rank = int(max_rank)
        self.count = 0

    def rank(self, s):
        if len(s) == 0 or s[0] == 0.0:
            return 0
        k = int(np.count_nonzero(s > self.eps * s[0]))
        if self.max_rank > 0:
            k = min(k, self.max_rank)
        return k

    def __call__(self, X, Y):
        """Best rank-k approximation of X Y^T under the rule: QR of both
        factors, SVD of R_X R_Y^T, keep the leading triplets."""
        self.count += 1
        m, K = X.shape
        n = Y.shape[0]
        if K == 0 or m == 0 or n == 0:
            return np.zeros((m, 0)), np.zeros((n, 0))
        Qx, Rx = np.linalg.qr(X)
        Qy, Ry = np.linalg.qr(Y)
        try:
            U, s, Vt = np.linalg.svd(Rx @ Ry.T)
        except np.linalg.LinAlgError:
            # the divide-and-conquer driver can fail to converge; the same
            # SVD by the QR-iteration driver
            U, s, Vt = sla.svd(Rx @ Ry.T, lapack_driver="gesvd")
        k = self.rank(s)
        return Qx @ (U[:, :k] * s[:k]), Qy @ Vt[:k].T


class HMatrix:
    """An H-matrix on a block tree, filled from a sparse matrix in cluster order."""

    def __init__(self, structure, A_csr, trunc):
        self.structure = structure
        self.trunc = trunc
        self.N = structure.N
        perm = structure.perm
        Ap = A_csr[perm][:, perm].tocsr()        # P A P^T, cluster order
        self.root = HBlock(structure.block_root)
        self.nonzero_admissible = 0
        for b in self.root.leaves():
            sub = Ap[b.r0:b.r1, b.c0:b.c1]
            if b.kind == DENSE:
                b.D = sub.toarray()
            else:
                # Algorithm 1, step I.  Admissible blocks of the sparse matrix
                # are normally empty; any entry found is kept by a truncated SVD.
                if sub.nnz and np.any(sub.data != 0.0):
                    self.nonzero_admissible += 1
                    b.X, b.Y = trunc(sub.toarray(), np.eye(b.n))
                else:
                    b.X, b.Y = np.zeros((b.m, 0)), np.zeros((b.n, 0))

    # ------------------------------------------------------------------ views
    def to_dense(self, blk=None):
        blk = blk or self.root
        out = np.zeros((blk.m, blk.n))
        for b in blk.leaves():
            r, c = b.r0 - blk.r0, b.c0 - blk.c0
            out[r:r + b.m, c:c + b.n] = b.D if b.kind == DENSE else b.X @ b.Y.T
        return out

    def ranks(self):
        return [b.X.shape[1] for b in self.root.leaves() if b.kind == LOWRANK]

    def storage_entries(self):
        tot = 0
        for b in self.root.leaves():
            tot += b.D.size if b.kind == DENSE else b.X.size + b.Y.size
        return tot


# ---------------------------------------------------------------- products
def hmul(B, V):
    """B @ V for an H-block B (every leaf taken in full)."""
    if B.kind == DENSE:
        return B.D @ V
    if B.kind == LOWRANK:
        return B.X @ (B.Y.T @ V)
    out = np.zeros((B.m, V.shape[1]))
    for i in range(2):
        for j in range(2):
            s = B.sons[i][j]
            out[s.r0 - B.r0:s.r1 - B.r0] += hmul(s, V[s.c0 - B.c0:s.c1 - B.c0])
    return out


def hmulT(B, V):
    """B^T @ V for an H-block B."""
    if B.kind == DENSE:
        return B.D.T @ V
    if B.kind == LOWRANK:
        return B.Y @ (B.X.T @ V)
    out = np.zeros((B.n, V.shape[1]))
    for i in range(2):
        for j in range(2):
            s = B.sons[i][j]
            out[s.c0 - B.c0:s.c1 - B.c0] += hmulT(s, V[s.r0 - B.r0:s.r1 - B.r0])
    return out


def add_lowrank(C, X, Y, trunc):
    """C += X Y^T, truncating in every low-rank leaf of C."""
    if C.kind == DENSE:
        C.D += X @ Y.T
    elif C.kind == LOWRANK:
        C.X, C.Y = trunc(np.hstack([C.X, X]), np.hstack([C.Y, Y]))
    else:
        for i in range(2):
            for j in range(2):
                s = C.sons[i][j]
                add_lowrank(s, X[s.r0 - C.r0:s.r1 - C.r0], Y[s.c0 - C.c0:s.c1 - C.c0], trunc)


def gemm(C, A, B, trunc):
    """C -= A B in H-arithmetic; A is (rows C) x t, B is t x (cols C)."""
    if A.kind == LOWRANK:
        _case("lowrank*any")
        add_lowrank(C, -A.X, hmulT(B, A.Y), trunc)
    elif B.kind == LOWRANK:
        _case("any*lowrank")
        add_lowrank(C, -hmul(A, B.X), B.Y, trunc)
    elif A.kind == DENSE and B.kind == DENSE:
        if C.kind == DENSE:
            _case("dense*dense->dense")
            C.D -= A.D @ B.D
        else:
            _case("dense*dense->other")
            add_lowrank(C, -A.D, B.D.T, trunc)
    elif A.kind == DENSE:                       # B subdivided: rows of C form a leaf
        W = hmulT(B, A.D.T)                     # (A.D B)^T
        if C.kind == DENSE:
            _case("dense*sub->dense")
            C.D -= W.T
        else:
            _case("dense*sub->other")
            add_lowrank(C, -np.eye(A.m), W, trunc)
    elif B.kind == DENSE:                       # A subdivided: cols of C form a leaf
        W = hmul(A, B.D)
        if C.kind == DENSE:
            _case("sub*dense->dense")
            C.D -= W
        else:
            _case("sub*dense->other")
            add_lowrank(C, -W, np.eye(B.n), trunc)
    elif C.kind == SUB:
        _case("sub*sub->sub")
        for i in range(2):
            for j in range(2):
                for k in range(2):
                    gemm(C.sons[i][j], A.sons[i][k], B.sons[k][j], trunc)
    elif C.kind == LOWRANK:
        _case("sub*sub->lowrank")
        # Both factors subdivided, low-rank target: form the product on the
        # four quadrants as truncated low-rank blocks, then add them to C with
        # one more truncation.
        Xs, Ys = [C.X], [C.Y]
        for i in range(2):
            for j in range(2):
                q = _TempLowRank(A.sons[i][0].r0, A.sons[i][0].r1,
                                 B.sons[0][j].c0, B.sons[0][j].c1)
                for k in range(2):
                    gemm(q, A.sons[i][k], B.sons[k][j], trunc)
                Xp = np.zeros((C.m, q.X.shape[1]))
                Yp = np.zeros((C.n, q.Y.shape[1]))
                Xp[q.r0 - C.r0:q.r1 - C.r0] = q.X
                Yp[q.c0 - C.c0:q.c1 - C.c0] = q.Y
                Xs.append(Xp)
                Ys.append(Yp)
        C.X, C.Y = trunc(np.hstack(Xs), np.hstack(Ys))
    else:
        raise AssertionError("dense target with two subdivided factors")


class _TempLowRank:
    """A rank-0 low-rank block used as an accumulation target."""

    kind = LOWRANK

    def __init__(self, r0, r1, c0, c1):
        self.r0, self.r1, self.c0, self.c1 = r0, r1, c0, c1
        self.X = np.zeros((r1 - r0, 0))
        self.Y = np.zeros((c1 - c0, 0))

    @property
    def m(self):
        return self.r1 - self.r0

    @property
    def n(self):
        return self.c1 - self.c0


# ------------------------------------------------------- dense leaf kernels
def getrf_nopiv(D):
    """Unpivoted LU of a dense square block; returns L\\U packed (L unit)."""
    D = D.copy()
    m = D.shape[0]
    for p in range(m):
        if D[p, p] == 0.0:
            raise ZeroPivot(f"zero pivot at local index {p}")
        D[p + 1:, p] /= D[p, p]
        D[p + 1:, p + 1:] -= np.outer(D[p + 1:, p], D[p, p + 1:])
    return D


def solve_unit_lower(D, V):
    return sla.solve_triangular(D, V, lower=True, unit_diagonal=True)


def solve_upper(D, V):
    return sla.solve_triangular(D, V, lower=False)


def solve_upper_T(D, V):
    """U^{-T} V for the upper triangle U of D."""
    return sla.solve_triangular(D, V, lower=False, trans="T")


def solve_unit_lower_T(D, V):
    return sla.solve_triangular(D, V, lower=True, unit_diagonal=True, trans="T")


# ------------------------------------------------------ H-triangular solves
def hsolve_lower(Ld, V):
    """L^{-1} V, L the unit lower triangle of the diagonal block Ld."""
    if Ld.kind == DENSE:
        return solve_unit_lower(Ld.D, V)
    n0 = Ld.sons[0][0].m
    V0 = hsolve_lower(Ld.sons[0][0], V[:n0])
    V1 = V[n0:] - hmul(Ld.sons[1][0], V0)
    return np.vstack([V0, hsolve_lower(Ld.sons[1][1], V1)])


def hsolve_upper(Ud, V):
    """U^{-1} V, U the upper triangle of the diagonal block Ud."""
    if Ud.kind == DENSE:
        return solve_upper(Ud.D, V)
    n0 = Ud.sons[0][0].m
    V1 = hsolve_upper(Ud.sons[1][1], V[n0:])
    V0 = V[:n0] - hmul(Ud.sons[0][1], V1)
    return np.vstack([hsolve_upper(Ud.sons[0][0], V0), V1])


def hsolve_upper_T(Ud, V):
    """U^{-T} V (U^T is lower triangular)."""
    if Ud.kind == DENSE:
        return solve_upper_T(Ud.D, V)
    n0 = Ud.sons[0][0].m
    V0 = hsolve_upper_T(Ud.sons[0][0], V[:n0])
    V1 = V[n0:] - hmulT(Ud.sons[0][1], V0)
    return np.vstack([V0, hsolve_upper_T(Ud.sons[1][1], V1)])


# ------------------------------------------------------------ H-TRSM, H-LU
def trsm_lower(Ld, B, trunc):
    """B := L^{-1} B for the block B in the block row of the diagonal block Ld."""
    if B.kind == LOWRANK:
        B.X = hsolve_lower(Ld, B.X)
    elif B.kind == DENSE:
        B.D = hsolve_lower(Ld, B.D)
    else:
        for j in range(2):
            trsm_lower(Ld.sons[0][0], B.sons[0][j], trunc)
            gemm(B.sons[1][j], Ld.sons[1][0], B.sons[0][j], trunc)
            trsm_lower(Ld.sons[1][1], B.sons[1][j], trunc)


def trsm_upper(Ud, B, trunc):
    """B := B U^{-1} for the block B in the block column of the diagonal block Ud."""
    if B.kind == LOWRANK:
        B.Y = hsolve_upper_T(Ud, B.Y)
    elif B.kind == DENSE:
        B.D = hsolve_upper_T(Ud, B.D.T).T
    else:
        for i in range(2):
            trsm_upper(Ud.sons[0][0], B.sons[i][0], trunc)
            gemm(B.sons[i][1], B.sons[i][0], Ud.sons[0][1], trunc)
            trsm_upper(Ud.sons[1][1], B.sons[i][1], trunc)


def hlu(D, trunc):
    """In-place H-LU of the diagonal block D (Algorithm 1, step II)."""
    if D.kind == DENSE:
        D.D = getrf_nopiv(D.D)
        return
    hlu(D.sons[0][0], trunc)
    trsm_lower(D.sons[0][0], D.sons[0][1], trunc)      # U12 = L11^{-1} A12
    trsm_upper(D.sons[0][0], D.sons[1][0], trunc)      # L21 = A21 U11^{-1}
    gemm(D.sons[1][1], D.sons[1][0], D.sons[0][1], trunc)   # A22 -= L21 U12
    hlu(D.sons[1][1], trunc)


# ------------------------------------------------------ applying the factors
def apply_U(Ud, V):
    """U V for the upper triangle (diagonal included) of the factored block."""
    if Ud.kind == DENSE:
        return np.triu(Ud.D) @ V
    n0 = Ud.sons[0][0].m
    top = apply_U(Ud.sons[0][0], V[:n0]) + hmul(Ud.sons[0][1], V[n0:])
    return np.vstack([top, apply_U(Ud.sons[1][1], V[n0:])])


def apply_L(Ld, V):
    """L V for the unit lower triangle of the factored block."""
    if Ld.kind == DENSE:
        return np.tril(Ld.D, -1) @ V + V
    n0 = Ld.sons[0][0].m
    bot = hmul(Ld.sons[1][0], V[:n0]) + apply_L(Ld.sons[1][1], V[n0:])
    return np.vstack([apply_L(Ld.sons[0][0], V[:n0]), bot])


class HLU:
    """H-LU factorisation of A and its use as a preconditioner."""

    def __init__(self, structure, A_csr, eps, max_rank=0):
        self.structure = structure
        self.trunc = Truncation(eps, max_rank)
        self.H = HMatrix(structure, A_csr, self.trunc)
        self.perm = structure.perm
        self.A = A_csr
        self.factored = False

    def factor(self):
        hlu(self.H.root, self.trunc)
        self.factored = True
        return self

    def solve(self, r):
        """z = P^T U^{-1} L^{-1} P r  (Algorithm 1, step III)."""
        r = np.asarray(r, dtype=np.float64)
        vec = r.ndim == 1
        R = r.reshape(len(r), -1)
        y = hsolve_lower(self.H.root, R[self.perm])
        z = hsolve_upper(self.H.root, y)
        out = np.empty_like(z)
        out[self.perm] = z
        return out[:, 0] if vec else out

    def apply_LU(self, V):
        """L U V in cluster order."""
        return apply_L(self.H.root, apply_U(self.H.root, V))

    def factor_error(self, nprobe=8, seed=12345, storage=np.float64):
        """|| (L U - P A P^T) Omega ||_F / || P A P^T Omega ||_F, Omega standard
        normal N x nprobe from numpy's default_rng(seed).

        storage: every stored entry of the factors (dense leaves, low-rank
        factors) is first rounded to this type; np.float32 gives the error of
        the computed factors once stored in FP32 (the FP32 precision pattern
        stores the H-LU in FP32; the paper has no FP32 mode).  The factors
        themselves are left unchanged."""
        Om = np.random.default_rng(seed).standard_normal((self.H.N, nprobe))
        Ap = self.A[self.perm][:, self.perm]
        ref = Ap @ Om
        saved = []
        if storage is not np.float64:
            for b in self.H.root.leaves():
                saved.append((b, b.D, b.X, b.Y))
                b.D = None if b.D is None else b.D.astype(storage).astype(np.float64)
                b.X = None if b.X is None else b.X.astype(storage).astype(np.float64)
                b.Y = None if b.Y is None else b.Y.astype(storage).astype(np.float64)
        try:
            return float(np.linalg.norm(self.apply_LU(Om) - ref) / np.linalg.norm(ref))
        finally:
            for b, D, X, Y in saved:
                b.D, b.X, b.Y = D, X, Y
