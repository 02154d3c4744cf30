"""Pins for the oracle's mesh and sparsity pattern (mesh of Example 1, Sec. 4)."""
import json
import os
from itertools import combinations

import numpy as np
import pytest

from oracle.assemble import Discretisation
from oracle.mesh import KuhnMesh

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def e_total(n):
    return 7 * n ** 3 + 9 * n ** 2 + 3 * n


def e_int(n):
    return 7 * n ** 3 - 9 * n ** 2 + 3 * n


@pytest.mark.parametrize("n", [1, 2, 3, 4, 6])
def test_counts_closed_form(n):
    m = KuhnMesh(n)
    assert len(m.tets) == 6 * n ** 3
    assert len(m.edges) == e_total(n)
    assert m.num_dofs == e_int(n)
    assert len(m.interior_vertices()) == (n - 1) ** 3
    # Euler characteristic of the ball: V - E + F - T = 1
    faces = set()
    for t in m.tets:
        for f in combinations(sorted(int(v) for v in t), 3):
            faces.add(f)
    assert (n + 1) ** 3 - len(m.edges) + len(faces) - len(m.tets) == 1


def test_table1_ndof_rows():
    """Total edge counts against the N_dof column the paper prints."""
    g = json.load(open(os.path.join(GOLDEN, "table1_ndof.json")))
    for k in g["exact_rows"]:
        assert e_total(2 ** (k - 1)) == g["printed"][str(k)]
    for k in (2, 3):                      # small enough to build the mesh
        assert len(KuhnMesh(2 ** (k - 1)).edges) == g["printed"][str(k)]


@pytest.mark.parametrize("n", [1, 2, 4])
def test_volumes_sum_to_one(n):
    d = Discretisation(n, 1.0)
    assert abs(d.volumes.sum() - 1.0) < 1e-14
    assert np.all(d.volumes > 0)
    assert np.allclose(d.volumes, 1.0 / (6 * n ** 3), rtol=0, atol=1e-15)


def _in_one_kuhn_tet(points):
    """Brute-force characterisation independent of the tet list: a point set
    lies in one Kuhn tetrahedron iff it is a chain for the componentwise
    order whose extent is at most one cell in every direction."""
    pts = sorted({tuple(p) for p in points}, key=lambda p: (sum(p), p))
    for a, b in zip(pts, pts[1:]):
        if any(x > y for x, y in zip(a, b)):
            return False
    lo, hi = np.array(pts[0]), np.array(pts[-1])
    return bool(np.all(hi - lo <= 1))


@pytest.mark.parametrize("n", [2, 3])
def test_pattern_brute_force(n):
    m = KuhnMesh(n)
    d = Discretisation(n, 1.0)
    e = m.interior_edges
    c = m.coords
    N = len(e)
    dense = np.zeros((N, N), dtype=bool)
    for i in range(N):
        for j in range(N):
            dense[i, j] = _in_one_kuhn_tet([c[e[i, 0]], c[e[i, 1]], c[e[j, 0]], c[e[j, 1]]])
    pat = d.A.copy()
    pat.data[:] = 1
    assert np.array_equal(pat.toarray().astype(bool), dense)


def test_pattern_counts():
    # nnz per mesh size (counted independently by a separate throwaway
    # enumeration when the workloads were sized): n=4: 3,916; n=8: 43,688.
    assert Discretisation(4, 1.0).A.nnz == 3916
    assert Discretisation(8, 1.0).A.nnz == 43688


def test_edge_orientation_and_order():
    m = KuhnMesh(3)
    e = m.edges
    assert np.all(e[:, 0] < e[:, 1])
    assert np.all(np.diff(e[:, 0] * 10 ** 6 + e[:, 1]) > 0)
    # every edge direction is one of the 7 Kuhn directions
    d = m.coords[e[:, 1]] - m.coords[e[:, 0]]
    assert np.all((d == 0) | (d == 1))
    assert np.all(d.sum(axis=1) >= 1)
    # midpoints are unique
    mid = m.midpoints2()
    assert len({tuple(x) for x in mid}) == len(mid)


@pytest.mark.parametrize("n", [1, 2, 3, 5])
def test_support_boxes_closed_form(n):
    """The edge from p to p + d (d a 0/1 vector on the Kuhn lattice) lies in
    the cubes with corner c, c_a = p_a where d_a = 1 and c_a in {p_a - 1, p_a}
    where d_a = 0 (both exist for an interior edge), and every tetrahedron's
    bounding box is its whole cube; so the support box is [p_a, p_a + 1] along
    the edge's axes and [p_a - 1, p_a + 1] across them."""
    m = KuhnMesh(n)
    lo, hi = m.support_boxes2()
    p = m.coords[m.interior_edges[:, 0]]
    d = m.coords[m.interior_edges[:, 1]] - p
    assert np.all((d == 0) | (d == 1))
    assert np.array_equal(lo, 2 * np.where(d == 1, p, p - 1))
    assert np.array_equal(hi, 2 * (p + 1))
    mid = m.midpoints2()
    assert np.all(lo <= mid) and np.all(mid <= hi)
    assert lo.min() >= 0 and hi.max() <= 2 * n


def _euler(m):
    V = len(np.unique(m.tets))
    F = len({tuple(sorted(int(t[a]) for a in range(4) if a != s)) for t in m.tets for s in range(4)})
    return V - len(m.edges) + F - len(m.tets)


@pytest.mark.parametrize("mm", [1, 2])
def test_two_box_domain_topology(mm):
    """The two-box domain (union of two crossing boxes, Example 2 read on the
    lattice): contractible, so V - E + F - T = 1; the union has 32 m^3 of the
    64 m^3 lattice cubes (a 4x3x2 and a 2x2x4 box, overlapping in 2x2x2)."""
    from paper_2211_11303_amd.inputs import two_box_mask
    n, mask = two_box_mask(mm)
    m = KuhnMesh(n, mask)
    assert int(mask.sum()) == 32 * mm ** 3 and len(m.tets) == 6 * 32 * mm ** 3
    assert _euler(m) == 1
    # every boundary edge lies on the boundary surface: both its ends are
    # boundary vertices
    bv = set(np.unique(m.tets).tolist()) - set(m.interior_vertices().tolist())
    for a, b in m.edges[~m.interior]:
        assert int(a) in bv and int(b) in bv


@pytest.mark.parametrize("n,m0,off", [(4, 2, (1, 0, 2)), (5, 3, (2, 1, 0)), (3, 3, (0, 0, 0))])
def test_cube_shaped_mask_is_a_scaled_cube(n, m0, off):
    """A mask that flags an m0^3 block of cubes at an offset gives the
    Kuhn mesh of the m0^3 cube: the same unknowns in the same order (the
    lattice shift keeps the vertex order), K scaled by n / m0 and M by m0 / n
    (lengths shrink by m0 / n; the Whitney forms grow like 1/h)."""
    from oracle.assemble import Discretisation
    mask = np.zeros(n ** 3, dtype=np.uint8)
    for k in range(off[2], off[2] + m0):
        for j in range(off[1], off[1] + m0):
            for i in range(off[0], off[0] + m0):
                mask[i + n * (j + n * k)] = 1
    dm = Discretisation(n, 1.0, mask=mask)
    dc = Discretisation(m0, 1.0)
    assert dm.N == dc.N == 7 * m0 ** 3 - 9 * m0 ** 2 + 3 * m0
    assert np.array_equal(dm.A.indptr, dc.A.indptr) and np.array_equal(dm.A.indices, dc.A.indices)
    sK, sM = n / m0, m0 / n
    assert abs(dm.K - sK * dc.K).max() <= 1e-13 * sK * abs(dc.K).max()
    assert abs(dm.M - sM * dc.M).max() <= 1e-13 * sM * abs(dc.M).max()
    shift = 2 * np.array(off)
    assert np.array_equal(dm.mesh.midpoints2(), dc.mesh.midpoints2() + shift)
