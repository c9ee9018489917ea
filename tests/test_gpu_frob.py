"""The Frobenius truncation rule (the paper's variant, eqn. curOff6) on the GPU
against the oracle.

N_i, the norm of all blocks of level i and below, is accumulated on the device
from the merged blocks of each level (the leaf level from the values of A); it
must equal the oracle's N_i to rounding (Frobenius norms do not see the
orthogonal changes of basis of the auxiliary variables).  Ranks must agree
(threshold ties replayed) and the FP64 stand-alone solve must match the
oracle's to 1e-10, for the small-block, large-block and RRQR compressions;
mixed precision reaches the GMRES tolerance.  The mean ranks of both rules at
the same epsilon are printed.
"""
import numpy as np
import pytest
import scipy.sparse as sp

import oracle
from parity_util import TOL, grid, oracle_matching, relerr

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def lx():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    torch.cuda.set_device(0)
    from paper_1510_07363_amd import lorax
    return lorax


@pytest.mark.parametrize("kind,nx,leaf,eps,method", [
    ("varcoef2d", 64, 64, 1e-4, "svd"),
    ("convdiff3d", 16, 64, 1e-3, "svd"),       # stacked blocks wider than 64 columns
    ("lognormal3d", 12, 32, 1e-5, "svd"),      # ragged leaves
    ("varcoef2d", 64, 64, 1e-5, "rrqr"),
])
def test_frob_rule_parity(lx, kind, nx, leaf, eps, method):
    csr, n, perm, lp, depth, rng = grid(kind, nx, leaf)
    F = lx.Factor(*csr, perm, lp, depth, eps, compress=method, rule="frob")
    Fo = oracle_matching(F, csr, perm, lp, depth, eps, method=method, rule="frob")
    st = F.stats()
    print("N_i gpu", {i: round(v, 6) for i, v in st["level_norm_by_level"].items()})
    print("N_i oracle", {i: round(v, 6) for i, v in Fo.level_norm.items()})
    for i in range(1, depth + 1):
        assert st["level_norm_by_level"][i] == pytest.approx(Fo.level_norm[i], rel=1e-11), i
    b = rng.uniform(-1, 1, (n, 2))
    x = F.solve(b)
    xo = np.column_stack([oracle.solve(Fo, b[:, k]) for k in range(2)])
    err = relerr(x, xo)
    Fc = lx.Factor(*csr, perm, lp, depth, eps, compress=method)
    print(f"{kind} {method}: solve vs oracle {err:.2e}; mean rank frob {st['mean_rank']:.2f} vs cutOff1 "
          f"{Fc.stats()['mean_rank']:.2f}; N_1 = {st['level_norm_by_level'][1]:.4e}")
    assert err <= TOL
    A = sp.csr_matrix((csr[2], csr[1], csr[0]), shape=(n, n))
    Fm = lx.Factor(*csr, perm, lp, depth, eps, compress=method, rule="frob", precision="mixed")
    xm, itm, rm = Fm.gmres(b, tol=TOL, restart=30, maxit=300)
    assert (np.linalg.norm(A @ xm - b, axis=0) / np.linalg.norm(b, axis=0) <= TOL).all()
