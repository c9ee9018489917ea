"""Pins of the oracle's cluster adjacency, well-separation and distance-2
colouring (Def. "adjacent clusters", Def. "distance of nodes", Cor.
"well-separated", Sec. 3) against a brute-force reading computed another way.

The brute force works on dense 0/1 matrices: the pattern P of A + A^T, and for
every partition level k the membership matrix L_k (2^k x n) whose row c marks
the original rows that tree positions of cluster c hold.  Cluster c and c' are
adjacent iff (L_k P L_k^T)[c, c'] > 0 with c != c', i.e. some unknown of c
couples to some unknown of c' in A.  Distances <= 2 come from the boolean
square of (I + adjacency).  None of this touches ClusterTree's leaf-pair
tables, so an over- or under-inclusive adjacency there (a wrong shift, a lost
direction of A, a level off by one) fails here.  Inputs are random sparse
patterns (not grids: unsymmetric entries, long-range couplings) on random
permutations and uneven leaf sizes.
"""
import numpy as np
import pytest

import oracle


def _random_problem(seed, n, depth, density):
    rng = np.random.default_rng(seed)
    # random unsymmetric pattern with a diagonal, plus a few long-range entries
    P = rng.random((n, n)) < density
    np.fill_diagonal(P, True)
    rows, cols = np.nonzero(P)
    row_ptr = np.zeros(n + 1, dtype=np.int64)
    np.add.at(row_ptr, rows + 1, 1)
    row_ptr = np.cumsum(row_ptr)
    col_idx = cols.astype(np.int32)            # np.nonzero is row-major, columns sorted
    perm = rng.permutation(n).astype(np.int32)
    nleaf = 1 << depth
    # uneven non-empty leaves
    cuts = np.sort(rng.choice(np.arange(1, n), nleaf - 1, replace=False))
    leaf_ptr = np.concatenate([[0], cuts, [n]]).astype(np.int32)
    return row_ptr, col_idx, perm, leaf_ptr, P


def _membership(perm, leaf_ptr, depth, k, n):
    L = np.zeros((1 << k, n), dtype=np.int64)
    per = 1 << (depth - k)
    for c in range(1 << k):
        t0, t1 = leaf_ptr[c * per], leaf_ptr[(c + 1) * per]
        L[c, perm[t0:t1]] = 1
    return L


@pytest.mark.parametrize("seed,n,depth,density", [(1, 40, 3, 0.04), (2, 64, 4, 0.03), (3, 96, 5, 0.02),
                                                  (4, 33, 5, 0.05), (5, 80, 4, 0.0)])
def test_cluster_adjacency_brute_force(seed, n, depth, density):
    row_ptr, col_idx, perm, leaf_ptr, P = _random_problem(seed, n, depth, density)
    T = oracle.ClusterTree(row_ptr, col_idx, perm, leaf_ptr, depth)
    S = (P | P.T).astype(np.int64)
    for k in range(depth + 1):
        L = _membership(perm, leaf_ptr, depth, k, n)
        assert np.all(L.sum(axis=0) == 1)          # a partition of the unknowns
        C = (L @ S @ L.T) > 0
        np.fill_diagonal(C, False)
        m = 1 << k
        for c in range(m):
            assert T.neighbours(k, c) == set(np.nonzero(C[c])[0].tolist()), (k, c)
        # distance <= 2 from the boolean square of (I + C); well-separated is its complement
        I1 = C | np.eye(m, dtype=bool)
        D2 = (I1.astype(np.int64) @ I1.astype(np.int64)) > 0
        for c in range(m):
            assert T.within2(k, c) == set(np.nonzero(D2[c])[0].tolist()), (k, c)
            for d in range(m):
                assert T.distance_le(k, c, d, 0) == (c == d)
                assert T.distance_le(k, c, d, 1) == bool(I1[c, d])
                assert T.distance_le(k, c, d, 2) == bool(D2[c, d])
                # well-separated (Cor. "well-separated"): neither equal nor adjacent
                assert (not T.adjacent_or_equal(k, c, d)) == (not I1[c, d])


@pytest.mark.parametrize("seed", [6, 7, 8])
def test_colouring_valid_against_brute_force_distances(seed):
    row_ptr, col_idx, perm, leaf_ptr, P = _random_problem(seed, 72, 4, 0.03)
    T = oracle.ClusterTree(row_ptr, col_idx, perm, leaf_ptr, 4)
    S = (P | P.T).astype(np.int64)
    for k in range(1, 5):
        L = _membership(perm, leaf_ptr, 4, k, 72)
        C = (L @ S @ L.T) > 0
        m = 1 << k
        I1 = C | np.eye(m, dtype=bool)
        D2 = (I1.astype(np.int64) @ I1.astype(np.int64)) > 0
        col = T.colouring(k)
        for a in range(m):
            for b in range(m):
                if a != b and D2[a, b]:
                    assert col[a] != col[b], (k, a, b)
            # greedy in ascending index: colour a is the smallest not used by an earlier
            # cluster within distance 2
            used = {col[b] for b in range(a) if D2[a, b]}
            assert col[a] == min(set(range(m + 1)) - used)


def test_compress_candidates_are_well_separated_by_brute_force():
    """Every compression's candidates p_1..p_t belong to clusters of P_{i-1} that
    are neither s's cluster nor adjacent to it (brute-force adjacency), and every
    such non-eliminated neighbour of s is a candidate (Sec. 4.3)."""
    from paper_1510_07363_amd import workloads as w
    rng = np.random.default_rng(3)
    nx = 8
    row_ptr, col_idx, val = w.diffusion3d(np.exp(rng.standard_normal(nx ** 3)), (nx, nx, nx))
    n = len(row_ptr) - 1
    depth = w.tree_depth(n, 8)
    perm, leaf_ptr = w.rcb_tree(w.grid_coords((nx, nx, nx)), depth)
    P = np.zeros((n, n), dtype=bool)
    P[np.repeat(np.arange(n), np.diff(row_ptr)), col_idx] = True
    S = (P | P.T).astype(np.int64)
    F = oracle.factor(row_ptr, col_idx, val, perm, leaf_ptr, depth, 1e-3, check=False)
    adj = {}
    for k in range(depth + 1):
        L = _membership(perm, leaf_ptr, depth, k, n)
        C = (L @ S @ L.T) > 0
        adj[k] = C | np.eye(1 << k, dtype=bool)
    seen = 0
    for rec in F.compressions:
        i, j = rec.level, rec.j
        for cand in rec.candidates:
            # a candidate is a super-node s_j'^[i] or a red node of P_{i-1}: cluster j' of P_{i-1}
            kind, lev, idx = cand
            assert (kind == "s" and lev == i) or (kind == "r" and lev == i - 1), cand
            assert not adj[i - 1][j, idx], (rec.level, rec.j, cand)
            seen += 1
    assert seen > 0
