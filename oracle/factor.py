"""Algorithm 1 (factorization using the H-tree), plain FP64.

Notation follows the paper.  Nodes of the H-tree are tuples
    ('r', i, c)  red node of cluster c of P_i
    ('s', i, j)  super-node s_j^[i] = (red(i, 2j), red(i, 2j+1))       (Sec. 4.2)
    ('b', i, j)  black node b_j^[i], whose parent P(b_j^[i]) = red(i-1, j)  (Def. H-tree)
An interaction edge u -> v carries Mat(e_{u->v}), a dense block of shape
(|v|, |u|): rows are the equations of v, columns the variables of u (Def.
"adjacency graph": Mat(e_{v_i -> v_j}) = A_{j,i}).

Steps (Sec. 4):
  Initialize      leaf red nodes carry the clusters of P_l; edges are the dense
                  blocks A[C_q, C_p] of adjacent leaf clusters and the diagonal
                  blocks (Sec. 4.1, Def. H-tree).
  MergeRedNodes   super-node blocks are the 2x2 concatenation of red blocks,
                  Mat(r1_j -> r0_j') in the top-right (Sec. 4.2, merge equation).
  Compress(s)     stack the blocks to and from all well-separated neighbours
                  p_1..p_t, B = [A_1;..;A_t;B_1;..;B_t] with A_k = Mat(s->p_k) and
                  B_k^T = Mat(p_k->s) (eqn. lra); B ~ [R;Q] V^T; rewire edges:
                  P(b)->p_k: R_k, p_k->P(b): Q_k^T, s->b: V^T, b->s: V,
                  b->P(b) and P(b)->b: -I_r (Sec. 4.3 and its edge-update list).
  Eliminate(v)    block Gauss elimination: for every in-edge k->v and out-edge
                  v->q add -Mat(v->q) Mat(v->v)^{-1} Mat(k->v) to Mat(k->q),
                  creating the edge when absent (Sec. 2.2); v's edges are then
                  frozen as factor blocks (Sec. 4.4).

Readings where the paper leaves a choice:
  * truncation: keep sigma_k with sigma_k / sigma_0 >= epsilon (eqn. cutOff1),
    sigma_0 the largest singular value of this node's stacked B; sigma_0 = 0 or
    no well-separated neighbour gives rank 0; epsilon = 0 keeps every singular
    value (exact);
  * V carries no singular values: V has orthonormal columns (right singular
    vectors) and [R;Q] = B V, so B - [R;Q] V^T = B (I - V V^T);
  * compress='rrqr' (the rank-revealing QR option the paper lists among
    alternative low-rank methods in Sec. 7): column-pivoted Householder QR of
    B^T, i.e. pivoting over the rows of B (largest remaining norm, lowest index
    on ties, norms recomputed at every step); stop at the first k with
    ||R22||_F <= epsilon * |R11|, R11 the first pivot.  Then V = the first k
    columns of the orthogonal factor, and ||B - B V V^T||_2 = ||R22||_2 <=
    epsilon * ||B||_2 since |R11| <= ||B||_2;
  * both A_k and B_k are always stacked (no symmetric shortcut);
  * pivot blocks are factored by LU with partial pivoting inside the block
    (LAPACK getrf); an exactly zero pivot is an error;
  * order inside a level: 'colored' (distance-2 colouring, then j) or
    'natural' (j ascending, as printed in Algorithm 1).

Self-checks (check=True): the sparsity-preservation theorem (Sec. 5: no edge is
created between nodes at distance > 2; at elimination every edge of the pivot
is at distance <= 1), well-separated candidates are never black or eliminated
nodes, and the parent red node has no edge before its compression.

Parity: pinned by tests against dense solves at epsilon = 0 (exact), special
cases that reduce to block LU at any epsilon (depth 1; a 1-D chain in natural
order), the printed elimination formulas of Sec. 2.3, the 2-norm bound of
every compression recomputed with an independent SVD, symmetry of the solve
operator for symmetric A, and the paper's printed accuracy for 2-D Poisson at
epsilon = 1e-4.
"""
from __future__ import annotations

from collections import defaultdict
from dataclasses import dataclass, field

import numpy as np
import scipy.linalg as sla
import scipy.sparse as sp

from .htree import ClusterTree


class SingularPivot(ArithmeticError):
    pass


@dataclass
class Frozen:
    """Factor data of one eliminated node p (used by SolveL / SolveU)."""
    node: tuple
    size: int
    lu: tuple | None                       # scipy lu_factor of Mat(p->p)
    fwd: list = field(default_factory=list)   # [(q, Mat(p->q))], q eliminated later
    bwd: list = field(default_factory=list)   # [(k, Mat(k->p))], k eliminated later


@dataclass
class CompressionRecord:
    level: int
    j: int
    rows: int                 # height of the stacked B
    m: int                    # width of B (size of the super-node)
    rank: int
    sigma: np.ndarray         # svd: singular values of B; rrqr: ||R22^(k)||_F, k = 0..
    candidates: list          # the well-separated neighbours p_1..p_t
    B: np.ndarray | None = None
    V: np.ndarray | None = None


@dataclass
class Factorization:
    n: int
    depth: int
    epsilon: float
    order: str
    perm: np.ndarray
    leaf_ptr: np.ndarray
    events: list              # ('merge', i, [(s, r0, r1)]) | ('elim', Frozen)
    size: dict
    compressions: list
    order_index: dict         # node -> elimination position (Order(p))
    level_colours: dict       # i -> number of colours used
    rule: str = "cutoff1"     # truncation rule
    level_norm: dict = field(default_factory=dict)   # i -> N_i of eqn. curOff6 (rule 'frob')

    def ranks_by_level(self):
        out = defaultdict(list)
        for c in self.compressions:
            out[c.level].append(c.rank)
        return dict(out)

    def compression_ratio(self):
        """<rank>_level / <super-node size>_level (Sec. 6.2, compression ratio)."""
        out = {}
        by = defaultdict(list)
        for c in self.compressions:
            by[c.level].append(c)
        for lev, recs in by.items():
            ms = np.mean([c.m for c in recs])
            out[lev] = (np.mean([c.rank for c in recs]) / ms) if ms > 0 else 0.0
        return out


class _Graph:
    """Active part of the H-tree: nodes, sizes and interaction edges."""

    def __init__(self):
        self.mat = {}
        self.out = defaultdict(set)
        self.inn = defaultdict(set)
        self.size = {}

    def has(self, u, v):
        return (u, v) in self.mat

    def get(self, u, v):
        return self.mat[(u, v)]

    def put(self, u, v, M):
        assert M.shape == (self.size[v], self.size[u]), (u, v, M.shape)
        self.mat[(u, v)] = M
        self.out[u].add(v)
        self.inn[v].add(u)

    def add(self, u, v, M):
        if (u, v) in self.mat:
            self.mat[(u, v)] = self.mat[(u, v)] + M
        else:
            self.put(u, v, M.copy())

    def drop(self, u, v):
        del self.mat[(u, v)]
        self.out[u].discard(v)
        self.inn[v].discard(u)

    def remove_node(self, p):
        for q in list(self.out[p]):
            self.drop(p, q)
        for k in list(self.inn[p]):
            self.drop(k, p)
        self.out.pop(p, None)
        self.inn.pop(p, None)


def _key(node):
    return ({"r": 0, "s": 1, "b": 2}[node[0]], node[1], node[2])


def factor(row_ptr, col_idx, val, perm, leaf_ptr, depth, epsilon, order="colored",
           forced_ranks=None, check=True, keep_blocks=False, compress="svd", rule="cutoff1",
           symmetric=False):
    """Algorithm 1.  Inputs are a CSR matrix (0-based) and the cluster tree.

    compress:     'svd' (eqn. cutOff1, as in the paper's experiments), 'rrqr', or
                  'rand' (adaptive randomized range finder, rand_compress, on
                  the nonzero rows and columns of the stacked block when it has
                  at most RAND_LMAX nonzero columns; wider ones take 'svd'; every
                  V of the factorization then has each column's entry of largest
                  magnitude positive, so that the auxiliary variables, and with
                  them the sketches of later blocks, are defined uniquely).
    rule:         'cutoff1': keep sigma_k >= epsilon sigma_0 of each stacked block
                  (eqn. cutOff1; RRQR: ||R22||_F <= epsilon |R11|);
                  'frob': the paper's variant of eqn. curOff6: the smallest k
                  with ||B - B V_k V_k^T||_F < epsilon N_i, where N_i^2 is the sum
                  of squared Frobenius norms of all blocks of the current level
                  and of the levels below, each level's blocks taken when that
                  level starts (after MergeRedNodes); the leaf level's blocks are
                  the blocks of A, so N_l = ||A||_F.  RRQR: the first k with
                  ||R22||_F < epsilon N_i.
    symmetric:    the half stack of the symmetric case (Sec. 4.3, last paragraph):
                  for symmetric A, B_k = A_k, so B stacks only A_k = Mat(s->p_k)
                  (Mat(p_k->s)^T where the first is absent) and Q_k = R_k.  A must
                  be symmetric (checked).

    forced_ranks: optional {(level, j): rank} to replay ranks decided elsewhere.
    keep_blocks:  keep every stacked B and V in the compression records (tests).
    """
    if not (0.0 <= epsilon < 1.0):
        raise ValueError("epsilon must be in [0, 1)")
    if rule not in ("cutoff1", "frob"):
        raise ValueError(rule)
    if symmetric:
        As = sp.csr_matrix((np.asarray(val, dtype=np.float64), np.asarray(col_idx), np.asarray(row_ptr)),
                           shape=(len(row_ptr) - 1,) * 2)
        if (As != As.T).nnz:
            raise ValueError("symmetric=True needs a symmetric matrix")
    if int(depth) < 1:
        raise ValueError("depth must be >= 1 (the root cluster is never a leaf)")
    T = ClusterTree(row_ptr, col_idx, perm, leaf_ptr, depth)
    l = T.l
    n = T.n
    A = sp.csr_matrix((np.asarray(val, dtype=np.float64), np.asarray(col_idx),
                       np.asarray(row_ptr)), shape=(n, n))
    Ap = A[T.perm][:, T.perm].tocsr()          # tree order
    G = _Graph()

    # ------------------------------------------------------------ Initialize (Sec. 4.1)
    nleaf = 1 << l
    for c in range(nleaf):
        G.size[("r", l, c)] = int(T.leaf_ptr[c + 1] - T.leaf_ptr[c])
    for p in range(nleaf):
        p0, p1 = T.leaf_range(p)
        for q in sorted({p} | T.neighbours(l, p)):
            q0, q1 = T.leaf_range(q)
            blk = np.asarray(Ap[q0:q1, p0:p1].todense(), dtype=np.float64)
            G.put(("r", l, p), ("r", l, q), blk)

    events = []
    compressions = []
    order_index = {}
    level_colours = {}
    level_norm = {}           # i -> N_i (rule 'frob')
    norm2 = 0.0
    counter = 0

    def clus(node):
        # cluster of P_{i-1} that a node taking part in level i corresponds to
        kind, lev, idx = node
        if kind == "r":
            return idx          # red(i-1, k) -> k
        return idx              # s_j^[i], b_j^[i] -> j

    for i in range(l, 0, -1):
        k_part = i - 1          # all distances at this level are in P_{i-1}

        # -------------------------------------------------- MergeRedNodes (Sec. 4.2)
        active = {u for u, e in G.out.items() if e} | {u for u, e in G.inn.items() if e}
        if check:
            for u in active:
                assert u[0] == "r" and u[1] == i, ("unexpected active node", u)
        groups = []
        for j in range(1 << (i - 1)):
            s = ("s", i, j)
            r0, r1 = ("r", i, 2 * j), ("r", i, 2 * j + 1)
            G.size[s] = G.size[r0] + G.size[r1]
            groups.append((s, r0, r1))
        owner = {}
        for s, r0, r1 in groups:
            owner[r0] = (s, 0)
            owner[r1] = (s, G.size[r0])
        merged = {}
        for (u, v), M in list(G.mat.items()):
            su, ou = owner[u]
            sv, ov = owner[v]
            if (su, sv) not in merged:
                merged[(su, sv)] = np.zeros((G.size[sv], G.size[su]))
            merged[(su, sv)][ov:ov + G.size[v], ou:ou + G.size[u]] = M
        for u in list(active):
            G.remove_node(u)
        for (su, sv), M in merged.items():
            G.put(su, sv, M)
        events.append(("merge", i, groups))
        # N_i^2 = N_{i+1}^2 + squared Frobenius norms of this level's blocks (eqn. curOff6)
        norm2 += sum(float(np.sum(M * M)) for M in G.mat.values())
        level_norm[i] = float(np.sqrt(norm2))

        js, cols = T.level_order(i, order)
        level_colours[i] = (max(cols) + 1) if cols else 0

        for j in js:
            s = ("s", i, j)
            b = ("b", i, j)
            P = ("r", i - 1, j)
            # ------------------------------------------------ Compress (Sec. 4.3)
            if check:
                assert not G.out.get(P) and not G.inn.get(P), "parent red node already has edges"
            nbrs = (G.out[s] | G.inn[s]) - {s}
            cand = sorted([p for p in nbrs if not T.adjacent_or_equal(k_part, clus(p), j)], key=_key)
            if check:
                for p in cand:
                    assert p[0] in ("s", "r"), ("well-separated black node", p)
                    assert p not in order_index, "eliminated candidate"
            forced = None
            if forced_ranks is not None and (i, j) in forced_ranks:
                forced = int(forced_ranks[(i, j)])
            tau = epsilon * level_norm[i] if rule == "frob" else None
            rec = _compress(G, s, b, P, cand, epsilon, forced, keep_blocks, compress, tau, symmetric,
                            task=(i << 24) | j, canon_sign=compress == "rand")
            rec.level, rec.j = i, j
            compressions.append(rec)

            # ------------------------------------- Eliminate(s), Eliminate(b) (Sec. 4.4)
            for v in (s, b):
                fr = _eliminate(G, v, T, k_part, clus, check)
                order_index[v] = counter
                counter += 1
                events.append(("elim", fr))

    return Factorization(n, l, float(epsilon), order, T.perm.copy(), T.leaf_ptr.copy(),
                         events, dict(G.size), compressions, order_index, level_colours, rule, level_norm)


def rrqr_rows(B, epsilon, forced_rank=None, tau=None):
    """Column-pivoted Householder QR of B^T (pivots are rows of B), truncated at
    the first k with ||R22||_F <= epsilon |R11| (or, given tau, the first k with
    ||R22||_F < tau).  Returns (k, V, pivots, tails) with V (m x k) orthonormal,
    tails[k] = ||R22^(k)||_F."""
    X = np.array(B, dtype=np.float64).T.copy()          # m x M
    m, M = X.shape
    kmax = min(m, M)
    pivoted = np.zeros(M, dtype=bool)
    vs, betas, piv, tails = [], [], [], []
    r11 = 0.0
    k = 0
    while k < kmax:
        nrm2 = np.sum(X[k:, :] ** 2, axis=0)
        nrm2[pivoted] = 0.0
        T = float(np.sqrt(np.sum(nrm2)))
        tails.append(T)
        p = int(np.argmax(nrm2))                        # first index of the maximum
        if k == 0:
            r11 = float(np.sqrt(nrm2[p]))
        if forced_rank is not None:
            if k >= forced_rank:
                break
        elif tau is not None:
            if T < tau:
                break
        elif T == 0.0 or T <= epsilon * r11:
            break
        x = X[k:, p].copy()
        alpha = -np.copysign(np.sqrt(np.sum(x * x)), x[0])
        v = x
        v[0] -= alpha
        beta = float(v @ v)
        if beta > 0.0:
            X[k:, :] -= np.outer(v, (2.0 / beta) * (v @ X[k:, :]))
        vs.append(v)
        betas.append(beta)
        piv.append(p)
        pivoted[p] = True
        k += 1
    if k == kmax:
        tails.append(0.0)
    V = np.eye(m)[:, :k].copy()
    for t in range(k - 1, -1, -1):                      # V = H_1 ... H_k I[:, :k]
        if betas[t] > 0.0:
            V[t:, :] -= np.outer(vs[t], (2.0 / betas[t]) * (vs[t] @ V[t:, :]))
    return k, V, piv, tails


# ------------------------------------------------------------- randomized compression
# Randomized range finder (Sec. 7 lists randomized SVD among the low-rank methods
# the algorithm admits), with the draws taken from a counter-based generator so
# that any implementation reproduces them: SplitMix64 (Steele, Lea and Flood,
# "Fast splittable pseudorandom number generators", 2014), output of the state
# equal to the counter.  The sketch is a Rademacher (random sign) matrix: sign of
# the top bit of the output for counter (task << 34) + (row << 6) + column,
# task = (level << 24) | j.
_M64 = (1 << 64) - 1
RAND_L0, RAND_LMAX = 16, 64


def splitmix64(x):
    """SplitMix64 output for state x (the state is advanced by the golden gamma
    before mixing, as in the published generator)."""
    z = (int(x) + 0x9E3779B97F4A7C15) & _M64
    z = ((z ^ (z >> 30)) * 0xBF58476D1CE4E5B9) & _M64
    z = ((z ^ (z >> 27)) * 0x94D049BB133111EB) & _M64
    return z ^ (z >> 31)


def rademacher(task, rows, cols):
    """rows x cols matrix of +-1: entry (a, t) is +1 when the top bit of
    splitmix64((task << 34) + (a << 6) + t) is 0."""
    out = np.empty((rows, cols))
    for a in range(rows):
        for t in range(cols):
            h = splitmix64(((task << 34) + (a << 6) + t) & _M64)
            out[a, t] = -1.0 if (h >> 63) else 1.0
    return out


def rand_rank(sig, uncaptured2, eps):
    """Smallest k with sqrt(uncaptured2 + sum_{t >= k} sig_t^2) <= eps sig_0 (the
    Frobenius norm of the discarded part, an upper bound of its 2-norm), or None
    when even k = len(sig) does not qualify."""
    if len(sig) == 0 or sig[0] == 0.0:
        return 0 if uncaptured2 == 0.0 else None
    thr = eps * sig[0]
    t2 = uncaptured2
    if not (np.sqrt(t2) <= thr):
        return None
    r = len(sig)
    for k in range(len(sig) - 1, -1, -1):
        t2 += sig[k] * sig[k]
        if np.sqrt(t2) <= thr:
            r = k
        else:
            break
    return r


def rand_compress(B, epsilon, task, l0=RAND_L0, lmax=RAND_LMAX):
    """Adaptive randomized compression of the stacked block B (M x c).
    With l = min(c, l0) sketch columns: Y = B^T Omega (Omega the Rademacher
    M x l matrix of the task), Q = the orthonormal factor of Householder QR of Y
    (c x l), C = B Q, C = U S W^T; the uncaptured energy is ||B||_F^2 - sum S^2
    (0 when l = c: Q is then a basis of the whole column space).  The rank is
    rand_rank(S, uncaptured, eps): the fewest directions whose discarded part
    has Frobenius norm <= eps S_0 <= eps ||B||_2, so ||B - B V V^T||_2 <= eps
    ||B||_2 holds (a-posteriori check).  Accepted when that rank is below l, or
    l = c; otherwise l doubles.  Returns (r, V, S, l), or None when l would
    exceed lmax while c > lmax (the caller then takes the SVD)."""
    M, c = B.shape
    l = min(c, l0)
    nB2 = float(np.sum(B * B))
    while True:
        Om = rademacher(task, M, l)
        Y = B.T @ Om
        Q, _ = np.linalg.qr(Y)                       # Householder (LAPACK geqrf), reduced
        C = B @ Q
        _, S, Wt = np.linalg.svd(C, full_matrices=False)
        unc = 0.0 if l == c else max(0.0, nB2 - float(np.sum(S * S)))
        r = rand_rank(S, unc, epsilon)
        if l == c or (r is not None and r < l):
            if r is None:
                r = l
            return r, Q @ Wt[:r].T, S, l
        if 2 * l > lmax and c > lmax:
            return None
        l = min(c, 2 * l)


def _compress(G, s, b, P, cand, epsilon, forced_rank=None, keep_blocks=False,
              method="svd", tau=None, symmetric=False, task=0, canon_sign=False):
    """Compress(s): replace the well-separated edges of s by low-rank edges through
    its black node b and the parent red node P = P(b) (Sec. 4.3, eqn. lra,
    eqn. anterpol, eqn. interpol and the edge-update list)."""
    m = G.size[s]
    if cand and symmetric:                             # half stack: A_k only (B_k = A_k)
        B = np.vstack([G.get(s, p) if G.has(s, p) else
                       (G.get(p, s).T if G.has(p, s) else np.zeros((G.size[p], m))) for p in cand])
    elif cand:
        parts = []
        for p in cand:                                 # A_k = Mat(s -> p_k)
            parts.append(G.get(s, p) if G.has(s, p) else np.zeros((G.size[p], m)))
        for p in cand:                                 # B_k = Mat(p_k -> s)^T
            parts.append(G.get(p, s).T if G.has(p, s) else np.zeros((G.size[p], m)))
        B = np.vstack(parts)
    else:
        B = np.zeros((0, m))
    # the randomized range finder works on the nonzero part of B: the rows and
    # columns that are zero (variables of a candidate that s does not touch) take
    # no part in the draw, so the sketch does not depend on that padding; its row
    # index is the position among the nonzero rows, in stacking order
    nzr = np.any(B != 0.0, axis=1) if B.size else np.zeros(B.shape[0], dtype=bool)
    nzc = np.any(B != 0.0, axis=0) if B.size else np.zeros(m, dtype=bool)
    if method == "rand" and int(nzc.sum()) > RAND_LMAX:
        method = "svd"                                  # blocks wider than the widest sketch
    if method == "rand":
        Bz = B[nzr][:, nzc]
        res = rand_compress(Bz, epsilon, task) if Bz.size else (0, np.zeros((Bz.shape[1], 0)), np.zeros(0), 0)
        if res is None:
            method = "svd"
        else:
            r, Vz, sig, _ = res
            V = np.zeros((m, r))
            V[nzc] = Vz
            if forced_rank is not None and forced_rank != r:
                raise ValueError("rank replay is not supported for randomized compression")
    if method == "svd":
        if B.shape[0] > 0 and m > 0:
            _, sig, Vt = np.linalg.svd(B, full_matrices=False)
        else:
            sig, Vt = np.zeros(0), np.zeros((0, m))
        if forced_rank is not None:
            r = forced_rank
        elif tau is not None:
            # eqn. curOff6: smallest k whose discarded tail has Frobenius norm < tau
            # (tail_k^2 = sum of sigma_t^2 for t >= k); all of B when none does
            tail2 = np.concatenate([np.cumsum((sig ** 2)[::-1])[::-1], [0.0]])
            ok = np.nonzero(np.sqrt(tail2) < tau)[0]
            r = int(ok[0]) if len(ok) else len(sig)
        elif len(sig) == 0 or sig[0] == 0.0:
            r = 0
        else:
            r = int(np.count_nonzero(sig >= epsilon * sig[0]))   # eqn. cutOff1
        V = Vt[:r].T.copy()                           # m x r, orthonormal columns
    elif method == "rand":
        pass
    elif method == "rrqr":
        if B.shape[0] > 0 and m > 0:
            r, V, _, sig = rrqr_rows(B, epsilon, forced_rank, tau)
            sig = np.asarray(sig)                     # ||R22^(k)||_F for k = 0..r
        else:
            r, V, sig = 0, np.zeros((m, 0)), np.zeros(0)
    else:
        raise ValueError(method)
    if canon_sign and V.size:
        # the auxiliary variables of b and P are the columns of V, each defined up
        # to its sign; a randomized sketch of a later stacked block sees that sign
        # (a deterministic SVD does not), so each column is fixed with its entry of
        # largest magnitude positive (lowest row on exact ties)
        piv = np.argmax(np.abs(V), axis=0)
        V = V * np.where(V[piv, np.arange(V.shape[1])] < 0.0, -1.0, 1.0)
    RQ = B @ V                                         # [R_1;..;R_t;Q_1;..;Q_t]
    rec = CompressionRecord(0, 0, B.shape[0], m, r, sig, list(cand),
                            B.copy() if keep_blocks else None,
                            V.copy() if keep_blocks else None)
    for p in cand:                                     # remove s <-> p_k
        if G.has(s, p):
            G.drop(s, p)
        if G.has(p, s):
            G.drop(p, s)
    G.size[b] = r
    G.size[P] = r
    t = len(cand)
    offs = np.cumsum([0] + [G.size[p] for p in cand] * (1 if symmetric else 2))
    for k, p in enumerate(cand):
        G.put(P, p, RQ[offs[k]:offs[k + 1]].copy())             # Mat(P(b) -> p_k) = R_k
        q0 = k if symmetric else t + k                          # Q_k = R_k when symmetric
        G.put(p, P, RQ[offs[q0]:offs[q0 + 1]].T.copy())         # Mat(p_k -> P(b)) = Q_k^T
    G.put(s, b, V.T.copy())                            # Mat(s -> b) = V^T
    G.put(b, s, V.copy())                              # Mat(b -> s) = V
    G.put(b, P, -np.eye(r))                            # Mat(b -> P(b)) = -I_r
    G.put(P, b, -np.eye(r))                            # Mat(P(b) -> b) = -I_r
    return rec


def _eliminate(G, v, T, k_part, clus, check):
    """Block Gauss elimination of node v (Sec. 2.2)."""
    m = G.size[v]
    K = sorted(G.inn[v] - {v}, key=_key)
    Q = sorted(G.out[v] - {v}, key=_key)
    if check:
        for u in K + Q:
            assert T.distance_le(k_part, clus(u), clus(v), 1), ("pivot edge at distance > 1", v, u)
    fr = Frozen(v, m, None)
    if m > 0:
        S = G.get(v, v) if G.has(v, v) else np.zeros((m, m))
        lu, piv = sla.lu_factor(S, check_finite=False)
        if np.any(np.diag(lu) == 0.0):
            raise SingularPivot(f"exactly singular pivot block at {v}")
        fr.lu = (lu, piv)
        W = {k: sla.lu_solve((lu, piv), G.get(k, v), check_finite=False) for k in K}
        for q in Q:
            Mq = G.get(v, q)
            for k in K:
                if check and not G.has(k, q):
                    assert T.distance_le(k_part, clus(k), clus(q), 2), ("fill at distance > 2", k, q)
                G.add(k, q, -(Mq @ W[k]))
    fr.fwd = [(q, G.get(v, q)) for q in Q]
    fr.bwd = [(k, G.get(k, v)) for k in K]
    G.remove_node(v)
    return fr
