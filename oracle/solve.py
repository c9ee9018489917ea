"""Algorithms 2-4 (solve with the hierarchical factorization), plain FP64.

  SetRHS     leaf red nodes take the entries of b of their cluster (tree order);
             every other red and black node starts from 0 (eqn. rhszero).
  forward    nodes in elimination order: SolveL(p): f = Mat(p->p)^{-1} RHS(p),
             then RHS(q) -= Mat(p->q) f for every out-edge to a node eliminated
             later (Algorithm 3).  Super-node right-hand sides are the
             concatenation of their red nodes' (eqn. concatRHS) when the level
             is merged.
  backward   nodes in reverse order: SolveU(p): Var(p) = RHS(p) - sum over
             in-edges from later nodes of Mat(q->p) Var(q), then
             Var(p) = Mat(p->p)^{-1} Var(p) (Algorithm 4); SplitVar hands the
             two halves of a super-node's variables to its red nodes
             (eqn. concatX).
The output is the concatenation of the leaf red nodes' variables, mapped back
from tree order to the original order.

Parity: pinned by tests (exactness at epsilon = 0 against a dense solve; the
special cases listed in the factor module; linearity and symmetry of the
operator).
"""
from __future__ import annotations

import numpy as np
import scipy.linalg as sla

from .factor import Factorization


def solve(F: Factorization, b):
    """x ~ A^{-1} b for b of shape (n,) or (n, nrhs) in the original ordering."""
    b = np.asarray(b, dtype=np.float64)
    vec = b.ndim == 1
    B = b.reshape(F.n, -1)
    nrhs = B.shape[1]
    bt = B[F.perm]                                   # tree order
    l = F.depth
    rhs = {}
    # ---------------------------------------------------------------- SetRHS
    for c in range(1 << l):
        rhs[("r", l, c)] = bt[F.leaf_ptr[c]:F.leaf_ptr[c + 1]].copy()

    def get_rhs(p):
        if p not in rhs:
            rhs[p] = np.zeros((F.size[p], nrhs))
        return rhs[p]

    # ------------------------------------------------------------ forward (SolveL)
    for ev in F.events:
        if ev[0] == "merge":
            for s, r0, r1 in ev[2]:
                rhs[s] = np.vstack([get_rhs(r0), get_rhs(r1)])
            continue
        fr = ev[1]
        p = fr.node
        if fr.size == 0:
            continue
        f = sla.lu_solve(fr.lu, get_rhs(p), check_finite=False)
        for q, M in fr.fwd:
            if M.size:
                rhs[q] = get_rhs(q) - M @ f

    # ----------------------------------------------------------- backward (SolveU)
    var = {}
    for ev in reversed(F.events):
        if ev[0] == "merge":
            for s, r0, r1 in ev[2]:
                xs = var[s]
                m0 = F.size[r0]
                var[r0] = xs[:m0]
                var[r1] = xs[m0:]
            continue
        fr = ev[1]
        p = fr.node
        if fr.size == 0:
            var[p] = np.zeros((0, nrhs))
            continue
        y = get_rhs(p).copy()
        for k, M in fr.bwd:
            if M.size:
                y -= M @ var[k]
        var[p] = sla.lu_solve(fr.lu, y, check_finite=False)

    xt = np.vstack([var[("r", l, c)] for c in range(1 << l)])
    x = np.empty_like(xt)
    x[F.perm] = xt
    return x[:, 0] if vec else x
