"""Pins of the oracle's GMRES (Sec. 6.2) against textbook properties."""
import numpy as np
import scipy.sparse as sp
import scipy.sparse.linalg as spla

import oracle
from paper_1510_07363_amd import workloads as w


def test_finite_termination_small():
    # restart >= n: GMRES reaches the exact solution in at most n steps
    rng = np.random.default_rng(0)
    n = 20
    A = np.eye(n) * 3 + rng.standard_normal((n, n)) * 0.3
    b = rng.standard_normal(n)
    out = oracle.fgmres(A, lambda v: v, b, tol=1e-13, restart=30, maxit=30)
    assert out["converged"] and out["iters"] <= n
    assert np.linalg.norm(out["x"] - np.linalg.solve(A, b)) / np.linalg.norm(np.linalg.solve(A, b)) < 1e-11


def test_estimate_monotone_within_cycle():
    rng = np.random.default_rng(1)
    n = 60
    A = np.eye(n) * 2 + rng.standard_normal((n, n)) * 0.2
    b = rng.standard_normal(n)
    out = oracle.fgmres(A, lambda v: v, b, tol=1e-12, restart=60, maxit=60)
    h = out["history"][1:]   # Arnoldi estimates of the first cycle
    assert all(h[i + 1] <= h[i] * (1 + 1e-12) for i in range(len(h) - 2))


def test_preconditioned_c1_reaches_1e10():
    p = w.make_config("poisson2d_32")
    A = p.scipy()
    F = oracle.factor(p.row_ptr, p.col_idx, p.val, p.perm, p.leaf_ptr, p.depth, 1e-2)
    out = oracle.fgmres(A, lambda v: oracle.solve(F, v), p.rhs[:, 0], tol=1e-10, restart=30)
    assert out["converged"] and out["relres"] <= 1e-10
    xd = spla.spsolve(A.tocsc(), p.rhs[:, 0])
    # kappa(A) ~ 441 for the 32x32 Laplacian
    assert np.linalg.norm(out["x"] - xd) / np.linalg.norm(xd) <= 441 * 1e-10 * 10
    # with a near-exact preconditioner GMRES needs very few steps
    F2 = oracle.factor(p.row_ptr, p.col_idx, p.val, p.perm, p.leaf_ptr, p.depth, 1e-12)
    out2 = oracle.fgmres(A, lambda v: oracle.solve(F2, v), p.rhs[:, 0], tol=1e-10)
    assert out2["iters"] <= 2


def test_nonconvergence_reported():
    rng = np.random.default_rng(2)
    n = 40
    A = sp.diags([np.linspace(1, 1e4, n)], [0]).tocsr()
    b = rng.standard_normal(n)
    out = oracle.fgmres(A, lambda v: v, b, tol=1e-30, restart=5, maxit=3)
    assert not out["converged"] and out["iters"] == 3 and out["relres"] > 0
