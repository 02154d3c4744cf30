"""Kuhn-split cube mesh of the unit cube and its interior edges.

Test infrastructure (see the package header): plain and slow on purpose.

The paper's Example 1 (Sec. 4) uses the unit cube, a coarse mesh of six
tetrahedra refined uniformly.  We use the direct Kuhn split of an n x n x n
grid of cubes: every cube is cut into the six tetrahedra spanned by the
monotone lattice paths from its lowest to its highest corner.  This mesh is
quasi-uniform, Ciarlet-regular (no hanging nodes) and shape-regular, as
Sec. 2.1 requires.  The unknowns of the lowest-order Nedelec space with the
perfect-conductor condition E x n = 0 (eq. (4), Sec. 2.1) are the interior
edges: edges that do not lie in a boundary face plane.

Numbering conventions (the paper is silent on them):

* vertex (i, j, k), 0 <= i, j, k <= n, has id  i + (n+1) * (j + (n+1) * k)
  and coordinates (i, j, k) / n;
* an edge is oriented from its lower vertex id to its higher one;
* interior edges are numbered in lexicographic (tail id, head id) order.
"""

from itertools import permutations

import numpy as np


def vertex_id(n, i, j, k):
    return i + (n + 1) * (j + (n + 1) * k)


def vertex_coords(n):
    """Integer lattice coordinates of all (n+1)^3 vertices, indexed by id."""
    ids = np.arange((n + 1) ** 3)
    i = ids % (n + 1)
    j = (ids // (n + 1)) % (n + 1)
    k = ids // (n + 1) ** 2
    return np.stack([i, j, k], axis=1)


def tetrahedra(n, mask=None):
    """The Kuhn tetrahedra of all n^3 cubes (or of the cubes (i, j, k) with
    mask[i + n (j + n k)] set) as rows of 4 vertex ids.

    For the cube with lowest corner c and each permutation p of the axes the
    tetrahedron is {c, c + e_p0, c + e_p0 + e_p1, c + (1, 1, 1)}.  Along each
    row the ids increase, so local vertex order equals global order.
    """
    tets = []
    for k in range(n):
        for j in range(n):
            for i in range(n):
                if mask is not None and not mask[i + n * (j + n * k)]:
                    continue
                c = np.array([i, j, k])
                for p in permutations(range(3)):
                    v = [c.copy()]
                    cur = c.copy()
                    for ax in p:
                        cur = cur.copy()
                        cur[ax] += 1
                        v.append(cur)
                    tets.append([vertex_id(n, *x) for x in v])
    return np.array(tets, dtype=np.int64)


def all_edges(n, tets=None):
    """Sorted unique (tail, head) pairs of all mesh edges, tail < head."""
    if tets is None:
        tets = tetrahedra(n)
    pairs = set()
    for t in tets:
        for a in range(4):
            for b in range(a + 1, 4):
                pairs.add((int(t[a]), int(t[b])))
    return np.array(sorted(pairs), dtype=np.int64)


def is_boundary_edge(n, coords, tail, head):
    """An edge lies in the boundary iff both ends share a face plane
    x_a = 0 or x_a = n for some axis a."""
    pt, ph = coords[tail], coords[head]
    for a in range(3):
        if pt[a] == ph[a] and (pt[a] == 0 or pt[a] == n):
            return True
    return False


def boundary_triangles(tets):
    """The faces that belong to exactly one tetrahedron: the triangles of the
    domain's boundary surface (sorted vertex-id triples)."""
    count = {}
    for t in tets:
        for skip in range(4):
            f = tuple(int(t[a]) for a in range(4) if a != skip)
            count[f] = count.get(f, 0) + 1
    return sorted(f for f, c in count.items() if c == 1)


class KuhnMesh:
    """The mesh, its edges and the interior-edge unknowns.

    ``mask`` (n^3 flags, cube (i, j, k) at i + n (j + n k)): the domain is
    the union of the flagged cubes, e.g. the two boxes of Example 2 on the
    lattice; an edge is then a boundary edge if it lies on a triangle of the
    boundary surface (a face of exactly one tetrahedron), so that the
    perfect-conductor condition of eq. (4) removes it.  Without a mask the
    domain is the whole cube and the face-plane rule below gives the same
    edges."""

    def __init__(self, n, mask=None):
        if n < 1:
            raise ValueError("n must be >= 1")
        self.n = n
        self.mask = None if mask is None else np.asarray(mask, dtype=bool).reshape(-1)
        if self.mask is not None and len(self.mask) != n ** 3:
            raise ValueError("mask needs n^3 entries")
        self.coords = vertex_coords(n)            # integer lattice coords
        self.tets = tetrahedra(n, self.mask)      # (6 cubes, 4) vertex ids
        self.edges = all_edges(n, self.tets)      # (E, 2), lexicographic
        self.edge_index = {(int(a), int(b)): e for e, (a, b) in enumerate(self.edges)}
        if self.mask is None:
            interior = [not is_boundary_edge(n, self.coords, a, b) for a, b in self.edges]
            self._boundary_vertices = None
        else:
            bedges, bverts = set(), set()
            for f in boundary_triangles(self.tets):
                bverts.update(f)
                bedges.update({(f[0], f[1]), (f[0], f[2]), (f[1], f[2])})
            interior = [(int(a), int(b)) not in bedges for a, b in self.edges]
            self._boundary_vertices = bverts
        self.interior = np.array(interior, dtype=bool)
        self.interior_edges = self.edges[self.interior]   # (N, 2), lexicographic
        # global edge index -> interior dof index (or -1)
        self.dof_of_edge = -np.ones(len(self.edges), dtype=np.int64)
        self.dof_of_edge[self.interior] = np.arange(int(self.interior.sum()))

    @property
    def num_dofs(self):
        return int(self.interior.sum())

    def midpoints2(self):
        """Doubled integer midpoint coordinates p_tail + p_head of the
        interior edges (lattice units), shape (N, 3)."""
        e = self.interior_edges
        return self.coords[e[:, 0]] + self.coords[e[:, 1]]

    def support_boxes2(self):
        """Support of every interior edge's basis function as a box: the
        bounding box of the tetrahedra containing the edge (the Whitney form
        of an edge vanishes on every other tetrahedron), in doubled lattice
        units like midpoints2; returns (lo2, hi2), each (N, 3)."""
        N = self.num_dofs
        lo = np.full((N, 3), np.iinfo(np.int64).max, dtype=np.int64)
        hi = np.full((N, 3), np.iinfo(np.int64).min, dtype=np.int64)
        for t in self.tets:
            pts = 2 * self.coords[t]
            tlo, thi = pts.min(axis=0), pts.max(axis=0)
            for a in range(4):
                for b in range(a + 1, 4):
                    d = self.dof_of_edge[self.edge_index[(int(t[a]), int(t[b]))]]
                    if d >= 0:
                        lo[d] = np.minimum(lo[d], tlo)
                        hi[d] = np.maximum(hi[d], thi)
        return lo, hi

    def interior_vertices(self):
        """Ids of the domain's vertices not on its boundary, increasing."""
        if self.mask is not None:
            used = set(int(v) for v in np.unique(self.tets))
            return np.array(sorted(used - self._boundary_vertices), dtype=np.int64)
        c = self.coords
        mask = np.all((c > 0) & (c < self.n), axis=1)
        return np.nonzero(mask)[0]
