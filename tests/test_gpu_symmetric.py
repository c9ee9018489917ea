"""The half stack of the symmetric case (Sec. 4.3, last paragraph) on the GPU.

For symmetric A the blocks B_k equal A_k, so Compress stacks only the A_k
(half the rows) and takes Q_k = R_k.  Bar: ranks equal the oracle's half-stack
ranks (ties replayed) and the FP64 stand-alone solve matches the oracle's to
1e-10, for small and large stacked blocks and RRQR; the result also matches the
GPU's own full-stack factorization (the full stack [A; A] only scales the
singular values by sqrt 2) to the same bar when the ranks agree; the
compression does less work (half the QR of the stacked block); mixed precision reaches the GMRES tolerance; a matrix that is not
symmetric is rejected with LRX_EINVAL.
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
    ("lognormal3d", 16, 64, 1e-4, "svd"),      # stacked blocks wider than 64 columns
    ("lognormal2d", 40, 16, 1e-4, "svd"),
    ("varcoef2d", 64, 64, 1e-5, "rrqr"),
])
def test_half_stack_parity(lx, kind, nx, leaf, eps, method):
    csr, n, perm, lp, depth, rng = grid(kind, nx, leaf)
    F = lx.Factor(*csr, perm, lp, depth, eps, compress=method, symmetric=True)
    Fo = oracle_matching(F, csr, perm, lp, depth, eps, method=method, symmetric=True)
    b = rng.uniform(-1, 1, (n, 2))
    x = F.solve(b)
    xo = np.column_stack([oracle.solve(Fo, b[:, k]) for k in range(2)])
    Ff = lx.Factor(*csr, perm, lp, depth, eps, compress=method)
    xf = Ff.solve(b)
    sh, sf = F.stats(), Ff.stats()
    print(f"{kind} {method}: vs oracle {relerr(x, xo):.2e}, vs full stack {relerr(x, xf):.2e}; compress "
          f"flops half/full {sh['flops_by_op']['compress'] / sf['flops_by_op']['compress']:.2f}")
    assert relerr(x, xo) <= TOL
    if list(F.ranks()[0]) == list(Ff.ranks()[0]):
        assert relerr(x, xf) <= TOL
    # half the stacked rows: the QR of B halves (the Jacobi on the c x c triangle does not)
    assert sh["flops_by_op"]["compress"] < sf["flops_by_op"]["compress"]
    A = sp.csr_matrix((csr[2], csr[1], csr[0]), shape=(n, n))
    Fm = lx.Factor(*csr, perm, lp, depth, eps, compress=method, symmetric=True, precision="mixed")
    xm, itm, rm = Fm.gmres(b, tol=TOL, restart=30, maxit=300)
    assert (np.linalg.norm(A @ xm - b, axis=0) / np.linalg.norm(b, axis=0) <= TOL).all()


def test_half_stack_rejects_nonsymmetric(lx):
    csr, n, perm, lp, depth, rng = grid("convdiff2d", 32, 16)
    with pytest.raises(lx.LoraxError) as e:
        lx.Factor(*csr, perm, lp, depth, 1e-4, symmetric=True)
    assert e.value.status == lx.LRX_EINVAL
