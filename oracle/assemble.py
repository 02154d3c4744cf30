"""Galerkin matrix of the lowest-order Nedelec (first kind) edge element.

Test infrastructure (see the package header).

Sec. 2.1 defines the bilinear form of eq. (5),
    a(E, Phi) = <curl E, curl Phi> - kappa_paper <E, Phi>,     (beta = 1)
on the Nedelec space N_0(T) = {a + b x x} and the edge basis fixed by
sigma(Phi_i, e_j) = delta_ij, sigma being the tangential line integral along
the interior edge e_j.  The Galerkin matrix of eq. (8) is A_ij = a(Phi_i, Phi_j).

The basis function of the edge (a, b) inside a tetrahedron is the Whitney
form  phi_ab = lambda_a grad(lambda_b) - lambda_b grad(lambda_a): it lies in
N_0(T), its tangential integral along (a, b) is 1 and along the other five
edges 0, so it is the dual basis the paper prescribes.  Its curl is the
constant 2 grad(lambda_a) x grad(lambda_b).  Both element integrals are
computed exactly, using  int_T lambda_x lambda_y = |T| (1 + delta_xy) / 20.

The wave number follows the notation A = K - kappa^2 M, i.e. the paper's
kappa (eq. (4)) is kappa^2 here.
"""

import numpy as np
import scipy.sparse as sp

from .mesh import KuhnMesh

LOCAL_EDGES = [(0, 1), (0, 2), (0, 3), (1, 2), (1, 3), (2, 3)]


def element_geometry(mesh):
    """Volumes |T| and barycentric gradients g[t, a, :] of every tetrahedron."""
    x = mesh.coords[mesh.tets].astype(np.float64) / mesh.n   # (T, 4, 3)
    J = np.stack([x[:, 1] - x[:, 0], x[:, 2] - x[:, 0], x[:, 3] - x[:, 0]], axis=2)
    det = np.linalg.det(J)
    vol = np.abs(det) / 6.0
    Jinv = np.linalg.inv(J)                          # row a-1 = grad(lambda_a)
    g = np.empty_like(x)
    g[:, 1:, :] = Jinv
    g[:, 0, :] = -Jinv.sum(axis=1)
    return vol, g


def element_matrices(vol, g):
    """Exact local curl-curl (K) and mass (M) matrices, shape (T, 6, 6)."""
    T = len(vol)
    Kl = np.zeros((T, 6, 6))
    Ml = np.zeros((T, 6, 6))

    def I(x, y):
        return vol * (1.0 + (x == y)) / 20.0

    def dot(u, v):
        return np.einsum("ti,ti->t", u, v)

    for e, (a, b) in enumerate(LOCAL_EDGES):
        ca = np.cross(g[:, a], g[:, b])
        for f, (c, d) in enumerate(LOCAL_EDGES):
            cc = np.cross(g[:, c], g[:, d])
            Kl[:, e, f] = vol * 4.0 * dot(ca, cc)
            Ml[:, e, f] = (dot(g[:, b], g[:, d]) * I(a, c)
                           - dot(g[:, b], g[:, c]) * I(a, d)
                           - dot(g[:, a], g[:, d]) * I(b, c)
                           + dot(g[:, a], g[:, c]) * I(b, d))
    return Kl, Ml


def local_to_global_edges(mesh):
    """Global edge index of each local edge of each tetrahedron, (T, 6)."""
    idx = np.empty((len(mesh.tets), 6), dtype=np.int64)
    for t, tet in enumerate(mesh.tets):
        for e, (a, b) in enumerate(LOCAL_EDGES):
            idx[t, e] = mesh.edge_index[(int(tet[a]), int(tet[b]))]
    return idx


def cube_of_tet(mesh):
    """Cube index (i, j, k) of every tetrahedron: its first vertex is the
    lowest corner of the cube it was cut from."""
    return mesh.coords[mesh.tets[:, 0]]


class Discretisation:
    """K, M on all edges; A = K - kappa^2 M on interior edges (CSR, FP64).

    ``beta_box = (i0, j0, k0, i1, j1, k1)`` with ``beta_in``: the curl-curl
    term carries the coefficient beta (eq. (5) has beta = 1; Sec. 2.1 allows
    a piecewise constant one, e.g. a magnetic block as in Example 3) equal
    to ``beta_in`` on the tetrahedra of the cubes i0 <= i < i1, j0 <= j < j1,
    k0 <= k < k1 and 1 elsewhere, so K_ij = sum_T beta_T int_T curl Phi_i .
    curl Phi_j.  Only the values change; the pattern stays that of beta = 1.
    ``mask``: the domain as a union of cubes (KuhnMesh)."""

    def __init__(self, n, kappa, beta_box=None, beta_in=1.0, mask=None):
        self.mesh = KuhnMesh(n, mask)
        self.kappa = float(kappa)
        vol, g = element_geometry(self.mesh)
        self.volumes = vol
        Kl, Ml = element_matrices(vol, g)
        self.beta = np.ones(len(vol))
        if beta_box is not None:
            lo = np.asarray(beta_box[:3])
            hi = np.asarray(beta_box[3:])
            c = cube_of_tet(self.mesh)
            inside = np.all((c >= lo) & (c < hi), axis=1)
            self.beta[inside] = float(beta_in)
        Kl = Kl * self.beta[:, None, None]
        l2g = local_to_global_edges(self.mesh)
        E = len(self.mesh.edges)
        rows = np.repeat(l2g, 6, axis=1).ravel()
        cols = np.tile(l2g, (1, 6)).ravel()
        self.K_full = sp.coo_matrix((Kl.ravel(), (rows, cols)), shape=(E, E)).tocsr()
        self.M_full = sp.coo_matrix((Ml.ravel(), (rows, cols)), shape=(E, E)).tocsr()
        for m in (self.K_full, self.M_full):
            m.sum_duplicates()
            m.sort_indices()
        # K_full and M_full come from the same triplets, so they share one
        # pattern: all pairs of edges that meet in a tetrahedron.  A is formed
        # on that pattern (explicit zeros kept), then restricted to the
        # interior edges.
        assert np.array_equal(self.K_full.indptr, self.M_full.indptr)
        assert np.array_equal(self.K_full.indices, self.M_full.indices)
        A_full = self.K_full.copy()
        A_full.data = self.K_full.data - self.kappa ** 2 * self.M_full.data
        inner = np.nonzero(self.mesh.interior)[0]
        self.K = self.K_full[inner][:, inner].tocsr()
        self.M = self.M_full[inner][:, inner].tocsr()
        self.A = A_full[inner][:, inner].tocsr()
        self.A.sort_indices()
        self.N = len(inner)

    def load(self, J):
        """b_j = <J, Phi_j> over the interior edges for a constant field J:
        the right-hand side of the weak form and of the Galerkin system
        (Sec. 2.1; Example 1 takes J_S = (0, 0, 1)).  The integral of a
        barycentric coordinate over T is |T|/4, so tetrahedron T adds
        |T|/4 J.(grad lambda_b - grad lambda_a) to its local edge (a, b)."""
        J = np.asarray(J, dtype=np.float64)
        vol, g = element_geometry(self.mesh)
        l2g = local_to_global_edges(self.mesh)
        full = np.zeros(len(self.mesh.edges))
        for e, (a, b) in enumerate(LOCAL_EDGES):
            np.add.at(full, l2g[:, e], vol / 4.0 * ((g[:, b] - g[:, a]) @ J))
        return full[self.mesh.interior]

    def discrete_gradient(self):
        """G: interior edges x interior vertices, +1 at the head, -1 at the tail."""
        mesh = self.mesh
        iv = mesh.interior_vertices()
        col_of = {int(v): c for c, v in enumerate(iv)}
        rows, cols, vals = [], [], []
        for d, (a, b) in enumerate(mesh.interior_edges):
            if int(b) in col_of:
                rows.append(d); cols.append(col_of[int(b)]); vals.append(1.0)
            if int(a) in col_of:
                rows.append(d); cols.append(col_of[int(a)]); vals.append(-1.0)
        return sp.csr_matrix((vals, (rows, cols)), shape=(self.N, len(iv)))

    def csr_arrays(self):
        """(row_ptr int32, col int32, val float64) of A with sorted columns."""
        A = self.A
        return (A.indptr.astype(np.int32), A.indices.astype(np.int32),
                A.data.astype(np.float64))
