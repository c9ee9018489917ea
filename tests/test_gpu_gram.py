"""Compression of blocks of at most 64 columns through the FP64 Gram matrix
(lrx_tune compress_gram: 1 = mixed precision, the default; 2 = mixed and
FP64): R1 and the column order come from G = B^T B and a Cholesky factorization
with diagonal pivoting instead of the QR and QRCP of B; the LQ and one-sided
Jacobi follow as on the QR path.

FP64 with compress_gram = 2: every other step is the FP64 path.  G carries an
absolute error of about c u sigma_0^2, so sigma_k is off by about
c u sigma_0^2 / sigma_k and a kept direction near the cut by an angle of about
c u sigma_0^2 / (sigma_r^2 - sigma_{r+1}^2); the next blocks inherit that,
so the path is not held to the oracle at 1e-10 (the QR path is).  Checked: the
first compression with a non-empty stacked block (its inputs are exact on both
sides) has the oracle's spectrum within 20 c u sigma_0^2 / sigma_k + 1e-13
sigma_0 for every sigma_k at or above epsilon sigma_0 / 100; the stand-alone
solve's error against the exact solution is within 1.5x of the QR path's plus
1e-12 (the distance to the oracle's solution is printed: a rank decided
differently near the threshold moves it to the size of the approximation error
itself).

Mixed precision (the default use): the stacked blocks already carry the FP32
products of earlier eliminations, so the path is checked by FGMRES reaching the
1e-10 true residual in no more iterations (+2) than the FP32 QR path
(compress_gram = 0) on the same inputs.

Blocks of more than 64 columns take the same front end in their own kernels
(the Gram matrix on the matrix cores over 32 x 32 tiles, the pivoted Cholesky
in panels of 16 pivots with the trailing update on the matrix cores, then the
LQ, Q2 and Jacobi of the QR route; one work-group back end for c <= 192, block
Jacobi rounds beyond).  Such blocks only occur above the first non-empty colour
step, where both sides' inputs already carry epsilon-accurate approximations, so
in FP64 each of their spectra is held to the QR route's within epsilon sigma_0,
the cut is checked on the reported spectrum, and the solve against the exact
solution as above; the timing classes show that no block took the QR route, and
the stored shapes which kernel family each block went to.  Mixed precision: the
FGMRES check above.
"""
import numpy as np
import pytest
import scipy.sparse as sp

import oracle
from parity_util import TOL, grid, relerr

pytestmark = pytest.mark.gpu

CONFIGS = [
    ("varcoef2d", 64, 64, 1e-4),
    ("lognormal3d", 12, 32, 1e-5),
    ("convdiff2d", 48, 16, 1e-3),
]


@pytest.fixture(scope="module")
def lx():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    torch.cuda.set_device(0)
    from paper_1510_07363_amd import lorax
    return lorax


@pytest.mark.parametrize("kind,nx,leaf,eps", CONFIGS)
def test_gram_fp64_accuracy(lx, kind, nx, leaf, eps):
    csr, n, perm, lp, depth, rng = grid(kind, nx, leaf)
    print(f"[gram fp64] {kind} nx={nx} leaf={leaf} eps={eps}", flush=True)
    base = lx.tune_get()
    try:
        lx.tune_set(compress_gram=2)
        F = lx.Factor(*csr, perm, lp, depth, eps)
        lx.tune_set(compress_gram=0)
        Fq = lx.Factor(*csr, perm, lp, depth, eps)
        Fo = oracle.factor(*csr, perm, lp, depth, eps, check=False)
        r, lv, js = F.ranks()
        first = next(i for i, c in enumerate(Fo.compressions) if len(c.sigma) and c.sigma[0] > 0)
        c = Fo.compressions[first]
        assert (int(lv[first]), int(js[first])) == (c.level, c.j) and int(r[first]) == c.rank
        so = np.asarray(c.sigma)
        t = F.tails(first)
        k = min(so.size, t.size - 1)
        d = np.abs(t[1:1 + k] - so[:k]) / so[0]
        big = so[:k] >= 0.01 * eps * so[0]
        bound = 20 * (t.size - 1) * 1.1102230246251565e-16 * so[0] / so[:k] + 1e-13
        assert (d[big] <= bound[big]).all(), (d[big] / bound[big]).max()
        A = sp.csr_matrix((csr[2], csr[1], csr[0]), shape=(n, n))
        xt = rng.uniform(-1, 1, (n, 2))
        b = A @ xt
        x, xq = F.solve(b), Fq.solve(b)
        xo = np.column_stack([oracle.solve(Fo, b[:, q]) for q in range(2)])
        e, eq = relerr(x, xt), relerr(xq, xt)
        print(f"{kind}: first spectrum within {d[big].max():.1e} sigma_0; error vs exact gram {e:.3e} qr {eq:.3e}; "
              f"gram vs oracle {relerr(x, xo):.2e}; mean rank {F.stats()['mean_rank']:.2f} vs "
              f"{Fq.stats()['mean_rank']:.2f}")
        assert e <= 1.5 * eq + 1e-12
    finally:
        lx.tune_set(**base)


@pytest.mark.parametrize("kind,nx,leaf,eps", CONFIGS)
def test_gram_mixed_gmres(lx, kind, nx, leaf, eps):
    csr, n, perm, lp, depth, rng = grid(kind, nx, leaf)
    base = lx.tune_get()
    try:
        b = rng.uniform(-1, 1, (n, 2))
        A = sp.csr_matrix((csr[2], csr[1], csr[0]), shape=(n, n))
        lx.tune_set(compress_gram=1)
        F = lx.Factor(*csr, perm, lp, depth, eps, precision="mixed")
        x, it, rr = F.gmres(b, tol=TOL, restart=30, maxit=300)
        res = np.linalg.norm(A @ x - b, axis=0) / np.linalg.norm(b, axis=0)
        lx.tune_set(compress_gram=0)
        Fq = lx.Factor(*csr, perm, lp, depth, eps, precision="mixed")
        xq, itq, rq = Fq.gmres(b, tol=TOL, restart=30, maxit=300)
        print(f"{kind}: GMRES iterations gram {list(it)} vs FP32 QR {list(itq)}; mean rank "
              f"{F.stats()['mean_rank']:.2f} vs {Fq.stats()['mean_rank']:.2f}; true residual {res.max():.2e}")
        assert (res <= TOL).all()
        assert max(it) <= max(itq) + 2
    finally:
        lx.tune_set(**base)


LARGE = [
    ("convdiff3d", 16, 64, 1e-3),       # blocks of 65..128 columns: one work-group back end
    ("convdiff3d", 28, 64, 1e-3),       # up to 240 columns: split back end (and tall blocks)
]


def _variant(M, c):
    if c <= 64:
        return "small"
    if c > 192 or M * c >= 1000000:
        return "split"
    return "tall" if M * c >= 300000 else "medium"


@pytest.mark.parametrize("kind,nx,leaf,eps", LARGE)
def test_gram_large_fp64_accuracy(lx, kind, nx, leaf, eps):
    csr, n, perm, lp, depth, rng = grid(kind, nx, leaf)
    print(f"[gram large fp64] {kind} nx={nx} leaf={leaf} eps={eps}", flush=True)
    base = lx.tune_get()
    try:
        lx.tune_set(compress_gram=2, large_split_c=192)     # every back end exercised
        lx.timing_enable(["compress", "compress_gram"])
        lx.timing_read()
        F = lx.Factor(*csr, perm, lp, depth, eps)
        tm = lx.timing_read()
        lx.timing_enable([])
        assert tm["compress"]["launches"] == 0 and tm["compress_gram"]["launches"] > 0, tm
        lx.tune_set(compress_gram=0)
        Fq = lx.Factor(*csr, perm, lp, depth, eps)
        r = F.ranks()[0]
        # the blocks of c > 64 sit above the first non-empty colour step, so both
        # routes' inputs already carry epsilon-accurate approximations of earlier
        # blocks: each spectrum must match the QR route's (itself held to the
        # oracle by the large-block tests) to epsilon sigma_0 (a wrong row of R
        # moves it by the size of sigma), and the cut must hold on it
        worst, fam = 0.0, {"small": 0, "medium": 0, "tall": 0, "split": 0}
        for i in range(len(r)):
            t, tq = F.tails(i), Fq.tails(i)
            if t[0] > 0 and 1 + int(r[i]) < len(t):
                assert t[1 + int(r[i])] <= eps * t[0] * (1 + 1e-12)
            M, cc = F.shape(i)
            assert (M, cc) == Fq.shape(i)
            if M == 0 or cc <= 64 or not tq[0] > 0:    # (an empty block reports one value)
                continue
            assert cc == len(t) - 1 == len(tq) - 1
            fam[_variant(M, cc)] += 1
            d = np.max(np.abs(t[1:] - tq[1:])) / tq[0]
            assert d <= eps, (i, M, cc, d)
            worst = max(worst, d)
        assert fam["medium"] + fam["tall"] + fam["split"] >= 5, fam
        if nx >= 28:
            assert fam["split"] >= 5 and fam["tall"] >= 1, fam
        A = sp.csr_matrix((csr[2], csr[1], csr[0]), shape=(n, n))
        xt = rng.uniform(-1, 1, (n, 2))
        b = A @ xt
        x, xq = F.solve(b), Fq.solve(b)
        e, eq = relerr(x, xt), relerr(xq, xt)
        print(f"{kind}: blocks of c > 64 {fam} within {worst:.1e} sigma_0 of the QR route; error vs exact "
              f"gram {e:.3e} qr {eq:.3e}; mean rank {F.stats()['mean_rank']:.2f} vs {Fq.stats()['mean_rank']:.2f}")
        assert e <= 1.5 * eq + 1e-12
    finally:
        lx.timing_enable([])
        lx.tune_set(**base)


@pytest.mark.parametrize("kind,nx,leaf,eps", LARGE)
def test_gram_large_mixed_gmres(lx, kind, nx, leaf, eps):
    """Mixed precision, the default route for blocks of more than 64 columns."""
    csr, n, perm, lp, depth, rng = grid(kind, nx, leaf)
    print(f"[gram large mixed] {kind} nx={nx} leaf={leaf} eps={eps}", flush=True)
    base = lx.tune_get()
    try:
        b = rng.uniform(-1, 1, (n, 2))
        A = sp.csr_matrix((csr[2], csr[1], csr[0]), shape=(n, n))
        lx.tune_set(compress_gram=1)
        F = lx.Factor(*csr, perm, lp, depth, eps, precision="mixed")
        x, it, rr = F.gmres(b, tol=TOL, restart=30, maxit=300)
        res = np.linalg.norm(A @ x - b, axis=0) / np.linalg.norm(b, axis=0)
        lx.tune_set(compress_gram=0)
        Fq = lx.Factor(*csr, perm, lp, depth, eps, precision="mixed")
        xq, itq, rq = Fq.gmres(b, tol=TOL, restart=30, maxit=300)
        print(f"{kind}: GMRES iterations gram {list(it)} vs QR {list(itq)}; mean rank "
              f"{F.stats()['mean_rank']:.2f} vs {Fq.stats()['mean_rank']:.2f}; true residual {res.max():.2e}")
        assert (res <= TOL).all()
        assert max(it) <= max(itq) + 2
    finally:
        lx.tune_set(**base)
