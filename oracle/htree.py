"""Clusters, cluster adjacency, H-tree distance and per-level colouring.

Follows Sec. 3 of the paper:
  * nested partitionings P_0..P_l with 2^i clusters at level i, each cluster the
    union of two children (Def. "nested partitionings");
  * two clusters are adjacent iff some leaf descendant of one is adjacent to a
    leaf descendant of the other, leaf adjacency being a non-zero block of A in
    either direction (Def. "adjacent clusters", Def. "adjacency graph");
  * the distance of two nodes is the path length between the corresponding
    clusters in the adjacency graph of the coarser partitioning; well-separated
    means distance > 1 (Def. "distance of nodes", Cor. "well-separated").

The colouring is the reading taken here of the freedom of elimination order the
paper grants (Sec. 1, last paragraphs; Sec. 7): at each level the super-nodes
are greedily coloured (ascending cluster index, smallest free colour) so that
two clusters of one colour are at distance >= 3 in the adjacency graph of
P_{i-1}.  By the sparsity-preservation theorem (Sec. 5) such nodes never share
a neighbour, so they may be processed in any order, or together.

Parity: pinned by the tests through brute-force BFS on small graphs and by the
exactness of the whole factorization at epsilon = 0.
"""
from __future__ import annotations

import numpy as np


class ClusterTree:
    """Nested binary partitionings given by a permutation and leaf pointers.

    perm[t]     original row/column index at tree position t
    leaf_ptr[c] first tree position of leaf cluster c (2^depth + 1 entries)
    Cluster c of level k is the union of leaves [c*2^(l-k), (c+1)*2^(l-k)).
    """

    def __init__(self, row_ptr, col_idx, perm, leaf_ptr, depth):
        self.l = int(depth)
        self.perm = np.asarray(perm, dtype=np.int64)
        self.leaf_ptr = np.asarray(leaf_ptr, dtype=np.int64)
        n = len(self.perm)
        if len(self.leaf_ptr) != (1 << self.l) + 1:
            raise ValueError("leaf_ptr must have 2^depth + 1 entries")
        if np.any(np.diff(self.leaf_ptr) <= 0) or self.leaf_ptr[0] != 0 or self.leaf_ptr[-1] != n:
            raise ValueError("leaves must be non-empty and cover all rows")
        if not np.array_equal(np.sort(self.perm), np.arange(n)):
            raise ValueError("perm is not a permutation")
        self.n = n
        self.pos = np.empty(n, dtype=np.int64)
        self.pos[self.perm] = np.arange(n)
        # leaf cluster of every original row
        leaf_of_pos = np.repeat(np.arange(1 << self.l), np.diff(self.leaf_ptr))
        self.leaf_of_row = leaf_of_pos[self.pos]
        # leaf adjacency from the pattern of A (both directions)
        row_ptr = np.asarray(row_ptr)
        col_idx = np.asarray(col_idx)
        rows = np.repeat(np.arange(n), np.diff(row_ptr))
        a = self.leaf_of_row[rows]
        b = self.leaf_of_row[col_idx]
        pairs = np.unique(np.stack([np.minimum(a, b), np.maximum(a, b)], 1), axis=0)
        pairs = pairs[pairs[:, 0] != pairs[:, 1]]
        self._adj = {}
        for k in range(self.l + 1):
            sh = self.l - k
            pk = np.unique(np.stack([pairs[:, 0] >> sh, pairs[:, 1] >> sh], 1), axis=0)
            pk = pk[pk[:, 0] != pk[:, 1]]
            nb = [set() for _ in range(1 << k)]
            for x, y in pk:
                nb[int(x)].add(int(y))
                nb[int(y)].add(int(x))
            self._adj[k] = nb
        self._dist2 = {}

    # ---------------------------------------------------------------- queries
    def leaf_range(self, c):
        return int(self.leaf_ptr[c]), int(self.leaf_ptr[c + 1])

    def neighbours(self, k, c):
        """Clusters adjacent to cluster c of P_k (c excluded)."""
        return self._adj[k][c]

    def adjacent_or_equal(self, k, a, b):
        return a == b or b in self._adj[k][a]

    def within2(self, k, c):
        """Clusters at distance <= 2 from c in the adjacency graph of P_k (c included)."""
        key = (k, c)
        s = self._dist2.get(key)
        if s is None:
            s = {c} | self._adj[k][c]
            for x in self._adj[k][c]:
                s |= self._adj[k][x]
            self._dist2[key] = s
        return s

    def distance_le(self, k, a, b, d):
        """True iff the path length between clusters a and b of P_k is <= d (d in 0..2)."""
        if d >= 2:
            return b in self.within2(k, a)
        if d == 1:
            return self.adjacent_or_equal(k, a, b)
        return a == b

    def colouring(self, k):
        """Greedy distance-2 colouring of the clusters of P_k in ascending index.
        Returns colour[c]."""
        m = 1 << k
        col = [-1] * m
        for c in range(m):
            used = {col[x] for x in self.within2(k, c) if x != c and col[x] >= 0}
            t = 0
            while t in used:
                t += 1
            col[c] = t
        return col

    def level_order(self, i, order):
        """Processing order of the super-nodes s_j^[i], j in [0, 2^(i-1)).

        'natural': j ascending, as written in Algorithm 1.
        'colored': by (colour, j) with the distance-2 colouring of P_{i-1}.
        Returns (list of j, list of colour per position)."""
        m = 1 << (i - 1)
        if order == "natural":
            return list(range(m)), list(range(m))
        if order != "colored":
            raise ValueError(order)
        col = self.colouring(i - 1)
        js = sorted(range(m), key=lambda j: (col[j], j))
        return js, [col[j] for j in js]
