"""Restarted GMRES with the hierarchical solve as preconditioner (Sec. 6.2).

The paper solves the left-preconditioned system (A~ A x = A~ b, eqn.
GMRES_residual).  The reading taken here uses right
preconditioning in its flexible form (FGMRES: the preconditioned vectors z_j
are kept, x = x_0 + Z y), restart m, x_0 = 0, modified Gram-Schmidt and Givens
rotations; a cycle ends when the Arnoldi estimate of the residual reaches
tol * ||b||, then the true relative residual ||b - A x|| / ||b|| (eqn. accres)
decides whether to stop or restart.  Also reported: the paper's
left-preconditioned residual of the final x.

Parity: pinned by tests: finite termination (restart >= n on n <= 30 returns the
dense solution), monotone residual estimate inside a cycle, agreement of the
final x with a sparse direct solve within kappa(A) * tol.
"""
from __future__ import annotations

import numpy as np


def fgmres(A, M, b, tol=1e-10, restart=30, maxit=500):
    """A: object with A @ v (e.g. scipy CSR); M: callable z = M(v) (preconditioner).

    Returns dict(x, iters, relres, converged, history, prec_relres)."""
    b = np.asarray(b, dtype=np.float64)
    n = b.shape[0]
    x = np.zeros(n)
    bnorm = np.linalg.norm(b)
    hist = []
    if bnorm == 0.0:
        return dict(x=x, iters=0, relres=0.0, converged=True, history=hist, prec_relres=0.0)
    it = 0
    converged = False
    while True:
        r = b - A @ x
        beta = np.linalg.norm(r)
        relres = beta / bnorm
        hist.append(relres)
        if relres <= tol:
            converged = True
            break
        if it >= maxit:
            break
        V = np.zeros((restart + 1, n))
        Z = np.zeros((restart, n))
        H = np.zeros((restart + 1, restart))
        cs = np.zeros(restart)
        sn = np.zeros(restart)
        g = np.zeros(restart + 1)
        g[0] = beta
        V[0] = r / beta
        k = 0
        for j in range(restart):
            Z[j] = M(V[j])
            w = A @ Z[j]
            for i in range(j + 1):                      # modified Gram-Schmidt
                H[i, j] = np.dot(w, V[i])
                w = w - H[i, j] * V[i]
            H[j + 1, j] = np.linalg.norm(w)
            if H[j + 1, j] != 0.0:
                V[j + 1] = w / H[j + 1, j]
            for i in range(j):                          # previous rotations
                t = cs[i] * H[i, j] + sn[i] * H[i + 1, j]
                H[i + 1, j] = -sn[i] * H[i, j] + cs[i] * H[i + 1, j]
                H[i, j] = t
            den = np.hypot(H[j, j], H[j + 1, j])
            cs[j] = H[j, j] / den if den != 0.0 else 1.0
            sn[j] = H[j + 1, j] / den if den != 0.0 else 0.0
            H[j, j] = den
            H[j + 1, j] = 0.0
            g[j + 1] = -sn[j] * g[j]
            g[j] = cs[j] * g[j]
            it += 1
            k = j + 1
            hist.append(abs(g[j + 1]) / bnorm)
            if abs(g[j + 1]) <= tol * bnorm or it >= maxit or den == 0.0:
                break
        y = np.zeros(k)
        for i in range(k - 1, -1, -1):                  # back substitution
            y[i] = (g[i] - H[i, i + 1:k] @ y[i + 1:k]) / H[i, i]
        x = x + Z[:k].T @ y
    Mb = M(b)
    Mr = M(b - A @ x)
    prec = np.linalg.norm(Mr) / np.linalg.norm(Mb) if np.linalg.norm(Mb) > 0 else 0.0
    return dict(x=x, iters=it, relres=relres, converged=converged, history=hist,
                prec_relres=prec)
