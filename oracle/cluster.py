"""Cluster tree and eta-admissible block cluster tree.

Test infrastructure (see the package header).

Sec. 3 builds the H-matrix on a block partition P obtained from a clustering
of the index set, with low-rank blocks chosen by eta-admissibility; Sec. 4
uses a geometrically balanced cluster tree and eta = 2.  The paper leaves the
details to its references, so the rules are fixed here (all integer
arithmetic on doubled lattice midpoints c = p_tail + p_head):

* cluster tree: a cluster with at most ``leaf`` indices is a leaf.  Otherwise
  take the tight bounding box [lo, hi] of its midpoints, pick the axis with
  the largest extent hi - lo (ties: lowest axis), and split at the box centre:
  indices with 2 c_axis < lo_axis + hi_axis go to the first son, the rest to
  the second; the split is stable.  The permutation to cluster order is the
  concatenation of the leaves in tree order.
* admissibility of a block (tau, sigma): dist > 0 and
  min(diam(tau), diam(sigma)) <= eta * dist, diam being the Euclidean
  diagonal of the tight box and dist the Euclidean gap between the two boxes
  (compared in squares, exactly).  The box of a cluster is the tight box of
  its midpoints, or, when a box is given for every index (e.g. the support
  of its basis function, as Definition 1 measures clusters by the supports
  of their basis functions), the bounding box of its indices' boxes; the
  splitting above always uses the midpoints.
* block tree: from (root, root); an admissible block is a low-rank leaf;
  otherwise, if tau or sigma is a leaf cluster the block is a dense leaf;
  otherwise it splits into the four products of the sons.
"""

import numpy as np


class Cluster:
    __slots__ = ("begin", "end", "lo", "hi", "alo", "ahi", "sons", "level", "id")

    def __init__(self, begin, end, lo, hi, level):
        self.begin, self.end = begin, end
        self.lo, self.hi = lo, hi
        self.alo, self.ahi = lo, hi       # box of the admissibility test
        self.sons = []
        self.level = level
        self.id = -1

    @property
    def size(self):
        return self.end - self.begin

    @property
    def is_leaf(self):
        return not self.sons


def build_cluster_tree(mid2, leaf, boxes=None):
    """Return (root, perm, clusters in pre-order).

    ``perm[i]`` is the natural index of the i-th index in cluster order.
    ``boxes = (lo2, hi2)`` (N x 3 each): the boxes of the admissibility test.
    """
    mid2 = np.asarray(mid2, dtype=np.int64)
    N = len(mid2)
    perm = np.arange(N)
    clusters = []

    def rec(idx, begin, level):
        pts = mid2[idx]
        lo = pts.min(axis=0)
        hi = pts.max(axis=0)
        c = Cluster(begin, begin + len(idx), lo, hi, level)
        if boxes is not None:
            c.alo = np.asarray(boxes[0], dtype=np.int64)[idx].min(axis=0)
            c.ahi = np.asarray(boxes[1], dtype=np.int64)[idx].max(axis=0)
        c.id = len(clusters)
        clusters.append(c)
        if len(idx) <= leaf:
            perm[begin:begin + len(idx)] = idx
            return c
        ext = hi - lo
        ax = int(np.argmax(ext))          # first maximum = lowest axis on ties
        left_mask = 2 * pts[:, ax] < lo[ax] + hi[ax]
        left = idx[left_mask]
        right = idx[~left_mask]
        c.sons = [rec(left, begin, level + 1),
                  rec(right, begin + len(left), level + 1)]
        return c

    root = rec(np.arange(N), 0, 0)
    return root, perm, clusters


def diam2(c):
    d = c.ahi - c.alo
    return int(d @ d)


def dist2(a, b):
    gap = np.maximum(0, np.maximum(b.alo - a.ahi, a.alo - b.ahi))
    return int(gap @ gap)


def admissible(a, b, eta):
    d2 = dist2(a, b)
    if d2 == 0:
        return False
    return min(diam2(a), diam2(b)) <= eta * eta * d2


DENSE, LOWRANK, SUB = 0, 1, 2


class BlockNode:
    __slots__ = ("row", "col", "kind", "sons")

    def __init__(self, row, col, kind):
        self.row, self.col, self.kind = row, col, kind
        self.sons = None           # 2x2 list for SUB


def build_block_tree(root, eta):
    """Block cluster tree; returns (root block, list of leaf blocks in
    pre-order)."""
    leaves = []

    def rec(t, s):
        if admissible(t, s, eta):
            b = BlockNode(t, s, LOWRANK)
            leaves.append(b)
            return b
        if t.is_leaf or s.is_leaf:
            b = BlockNode(t, s, DENSE)
            leaves.append(b)
            return b
        b = BlockNode(t, s, SUB)
        b.sons = [[rec(t.sons[i], s.sons[j]) for j in range(2)] for i in range(2)]
        return b

    return rec(root, root), leaves


class Structure:
    """Cluster tree + block tree of one problem."""

    def __init__(self, mid2, leaf, eta=2.0, boxes=None):
        self.leaf = int(leaf)
        self.eta = float(eta)
        self.root, self.perm, self.clusters = build_cluster_tree(mid2, leaf, boxes)
        self.block_root, self.block_leaves = build_block_tree(self.root, eta)
        self.N = len(self.perm)

    def leaf_clusters(self):
        return [c for c in self.clusters if c.is_leaf]

    def summary(self):
        dense = [b for b in self.block_leaves if b.kind == DENSE]
        lr = [b for b in self.block_leaves if b.kind == LOWRANK]
        return {
            "clusters": len(self.clusters),
            "leaves": len(self.leaf_clusters()),
            "depth": max(c.level for c in self.clusters),
            "admissible": len(lr),
            "dense": len(dense),
            "dense_entries": sum(b.row.size * b.col.size for b in dense),
            "lowrank_rows_plus_cols": sum(b.row.size + b.col.size for b in lr),
        }
