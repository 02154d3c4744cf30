"""Pins for the oracle's cluster tree and block cluster tree (Sec. 3,
Definition 1; eta = 2 and the geometric cluster tree of Sec. 4)."""
import numpy as np
import pytest

from oracle.assemble import Discretisation
from oracle.cluster import DENSE, LOWRANK, SUB, Structure
from oracle.mesh import KuhnMesh


def _check_cluster_tree(s, mid2, leaf):
    N = len(mid2)
    assert sorted(s.perm.tolist()) == list(range(N))
    leaves = s.leaf_clusters()
    # leaves partition 0..N-1 in order, contiguous, and are small enough
    pos = 0
    for c in leaves:
        assert c.begin == pos and 0 < c.size <= leaf
        pos = c.end
    assert pos == N
    for c in s.clusters:
        pts = mid2[s.perm[c.begin:c.end]]
        assert np.array_equal(c.lo, pts.min(axis=0)) and np.array_equal(c.hi, pts.max(axis=0))
        if c.is_leaf:
            assert c.size <= leaf
            continue
        assert c.size > leaf
        a, b = c.sons
        assert a.begin == c.begin and a.end == b.begin and b.end == c.end
        ext = c.hi - c.lo
        ax = [i for i in range(3) if ext[i] == ext.max()][0]
        pa = mid2[s.perm[a.begin:a.end]][:, ax]
        pb = mid2[s.perm[b.begin:b.end]][:, ax]
        assert np.all(2 * pa < c.lo[ax] + c.hi[ax])
        assert np.all(2 * pb >= c.lo[ax] + c.hi[ax])
        # the split is stable: each son keeps the natural order of its parent
        order = {int(v): i for i, v in enumerate(s.perm[c.begin:c.end])}
        for son in (a, b):
            idx = [order[int(v)] for v in s.perm[son.begin:son.end]]
            assert idx == sorted(idx)


def _box_test(t, u, eta):
    gap = np.maximum(0, np.maximum(u.lo - t.hi, t.lo - u.hi)).astype(float)
    dist = float(np.sqrt(gap @ gap))
    dt = float(np.sqrt(((t.hi - t.lo) ** 2).sum()))
    du = float(np.sqrt(((u.hi - u.lo) ** 2).sum()))
    return dist > 0 and min(dt, du) <= eta * dist + 1e-9 * max(dt, du)


def _check_block_tree(s, eta, A_perm, expect_empty):
    N = s.N
    area = 0
    for b in s.block_leaves:
        area += b.row.size * b.col.size
        if b.kind == LOWRANK:
            assert b.row is not b.col
            assert _box_test(b.row, b.col, eta)
            # at the workload leaf sizes no entry of the sparse matrix falls
            # in an admissible block (tiny leaves can see neighbours as far)
            if expect_empty:
                sub = A_perm[b.row.begin:b.row.end, b.col.begin:b.col.end]
                assert sub.nnz == 0
        else:
            assert b.kind == DENSE
            assert b.row.is_leaf or b.col.is_leaf
            assert not _box_test(b.row, b.col, eta)
    assert area == N * N

    def walk(node, parent_adm):
        if node.kind == SUB:
            assert not _box_test(node.row, node.col, eta)
            for row in node.sons:
                for sn in row:
                    walk(sn, False)
    walk(s.block_root, False)
    # the diagonal is subdivided down to dense leaf blocks
    diag = [b for b in s.block_leaves if b.row is b.col]
    assert len(diag) == len(s.leaf_clusters())
    assert all(b.kind == DENSE for b in diag)


@pytest.mark.parametrize("n,leaf", [(4, 32), (4, 8), (5, 20), (6, 16), (8, 64)])
def test_structure_invariants(n, leaf):
    d = Discretisation(n, 1.0)
    mid2 = d.mesh.midpoints2()
    s = Structure(mid2, leaf, 2.0)
    _check_cluster_tree(s, mid2, leaf)
    _check_block_tree(s, 2.0, d.A[s.perm][:, s.perm].tocsr(), expect_empty=leaf >= 32)


def test_structure_counts_small():
    # Counts recorded when the workloads were sized (independent enumeration):
    # 4^3 cubes, leaf 32 -> 29 clusters, 15 leaves of 17..28 indices, depth 4,
    # 82 admissible and 129 dense blocks holding 65,262 entries.
    s = Structure(KuhnMesh(4).midpoints2(), 32, 2.0)
    sm = s.summary()
    assert (sm["clusters"], sm["leaves"], sm["depth"]) == (29, 15, 4)
    assert (sm["admissible"], sm["dense"], sm["dense_entries"]) == (82, 129, 65262)
    sizes = [c.size for c in s.leaf_clusters()]
    assert (min(sizes), max(sizes)) == (17, 28)


@pytest.mark.slow
def test_structure_counts_16():
    s = Structure(KuhnMesh(16).midpoints2(), 64, 2.0)
    sm = s.summary()
    assert (sm["clusters"], sm["leaves"], sm["depth"]) == (1021, 511, 9)
    assert (sm["admissible"], sm["dense"], sm["dense_entries"]) == (14824, 10623, 29829200)


def _box_test_union(s, t, u, eta, lo2, hi2):
    """Admissibility by brute force on the union of the indices' boxes."""
    it, iu = s.perm[t.begin:t.end], s.perm[u.begin:u.end]
    tl, th = lo2[it].min(axis=0), hi2[it].max(axis=0)
    ul, uh = lo2[iu].min(axis=0), hi2[iu].max(axis=0)
    gap = np.maximum(0, np.maximum(ul - th, tl - uh)).astype(float)
    dist = float(np.sqrt(gap @ gap))
    dt = float(np.sqrt(((th - tl) ** 2).sum()))
    du = float(np.sqrt(((uh - ul) ** 2).sum()))
    return dist > 0 and min(dt, du) <= eta * dist + 1e-9 * max(dt, du)


@pytest.mark.parametrize("n,leaf", [(4, 8), (4, 32), (6, 16), (8, 64)])
def test_support_box_structure(n, leaf):
    """Admissibility on the basis functions' supports (Definition 1 measures
    clusters by the supports): the cluster tree is the midpoint tree; the
    blocks pass or fail the brute-force test on the union of the supports;
    and, at every leaf size, no entry of A falls in an admissible block (two
    basis functions couple only if their supports meet)."""
    d = Discretisation(n, 1.0)
    mid2 = d.mesh.midpoints2()
    lo2, hi2 = d.mesh.support_boxes2()
    s = Structure(mid2, leaf, 2.0, boxes=(lo2, hi2))
    s0 = Structure(mid2, leaf, 2.0)
    _check_cluster_tree(s, mid2, leaf)
    assert np.array_equal(s.perm, s0.perm)
    Ap = d.A[s.perm][:, s.perm].tocsr()
    area = 0
    for b in s.block_leaves:
        area += b.row.size * b.col.size
        adm = _box_test_union(s, b.row, b.col, 2.0, lo2, hi2)
        assert adm == (b.kind == LOWRANK)
        if b.kind == LOWRANK:
            assert Ap[b.row.begin:b.row.end, b.col.begin:b.col.end].nnz == 0
        else:
            assert b.row.is_leaf or b.col.is_leaf
    assert area == s.N * s.N
    # a support box contains its midpoint, so a block admissible on the
    # supports is admissible on the midpoints (there or at an ancestor): the
    # dense area can only grow, and it does at these sizes
    assert s.summary()["dense_entries"] > s0.summary()["dense_entries"]


def test_support_box_special_case():
    """Point boxes (each index's box its own midpoint) reproduce the midpoint
    structure exactly."""
    mid2 = KuhnMesh(5).midpoints2()
    s = Structure(mid2, 20, 2.0, boxes=(mid2, mid2))
    s0 = Structure(mid2, 20, 2.0)
    assert [b.kind for b in s.block_leaves] == [b.kind for b in s0.block_leaves]
    assert [(b.row.id, b.col.id) for b in s.block_leaves] == [(b.row.id, b.col.id) for b in s0.block_leaves]
