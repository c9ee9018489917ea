"""GPU results against the FP64 oracle on the shapes the measured workloads run.

* The exact 2-D variable-coefficient workload (256 x 256, n = 65,536, leaf
  clusters of 64, epsilon = 1e-4): FP64 stand-alone solve parity with the
  oracle (rank replay on threshold ties) <= 1e-10; FGMRES(30) true residual
  <= 1e-10 in FP64 and mixed precision, with the mixed result's distance to the
  FP64 result inside the conditioning bound ||A^-1||_2 (||r|| + ||r_o||).
* The 3-D convection-diffusion recipe at the headline 3-D shape (leaf
  clusters of 128, epsilon = 1e-3) on a 32^3 grid: its stacked blocks take the
  large-block variants (more than 192 columns: panel QRs and block-Jacobi
  rounds; tall 64 < c <= 192 blocks: the panel tall QR), and the solution must
  match the oracle's to 1e-10 in FP64 (a wrong V in any variant would move the
  solution far beyond that: the solve is invariant only under orthogonal
  changes of basis of the same subspace).
* Batched factorization (several systems in one level loop) and served
  answers against the oracle, not only against the single-system calls.
"""
import numpy as np
import pytest
import scipy.sparse as sp
import scipy.sparse.linalg as spla

import oracle
from paper_1510_07363_amd import workloads as w
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


def _smin_bound(A, b, r1, r2):
    """||x1 - x2|| <= ||A^-1||_2 (||b - A x1|| + ||b - A x2||); ||A^-1||_2 from the
    smallest singular value, computed by a shift-invert Lanczos on A^T A."""
    n = A.shape[0]
    lu = spla.splu(A.tocsc())
    op = spla.LinearOperator((n, n), matvec=lambda v: lu.solve(lu.solve(v, trans="T")), dtype=np.float64)
    lam = spla.eigsh(op, k=1, which="LM", return_eigenvectors=False, tol=1e-6)[0]
    inv_norm = np.sqrt(lam)
    return inv_norm * (r1 + r2) * np.linalg.norm(b)


def test_varcoef2d_256_exact_config(lx):
    p = w.make_config("varcoef2d_256")
    csr = (p.row_ptr, p.col_idx, p.val)
    print(f"[c2] n={p.n} depth={p.depth} eps={p.epsilon}", flush=True)
    F = lx.Factor(*csr, p.perm, p.leaf_ptr, p.depth, p.epsilon)
    Fo = oracle_matching(F, csr, p.perm, p.leaf_ptr, p.depth, p.epsilon)
    b = p.rhs[:, :2]
    x = F.solve(b)
    xo = np.column_stack([oracle.solve(Fo, b[:, k]) for k in range(2)])
    err = relerr(x, xo)
    print(f"[c2] FP64 solve vs oracle: {err:.2e}", flush=True)
    assert err <= TOL
    A = p.scipy()
    xg, its, rr = F.gmres(p.rhs, tol=TOL, restart=30, maxit=500)
    res = np.linalg.norm(A @ xg - p.rhs, axis=0) / np.linalg.norm(p.rhs, axis=0)
    assert (res <= TOL).all() and (rr <= TOL).all()
    Fm = lx.Factor(*csr, p.perm, p.leaf_ptr, p.depth, p.epsilon, precision="mixed")
    xm, itm, rm = Fm.gmres(p.rhs, tol=TOL, restart=30, maxit=500)
    resm = np.linalg.norm(A @ xm - p.rhs, axis=0) / np.linalg.norm(p.rhs, axis=0)
    assert (resm <= TOL).all() and (rm <= TOL).all()
    assert (itm <= its + 2).all()
    # per-result error of the mixed answer against the oracle's FP64 FGMRES answer
    k = 0
    o = oracle.fgmres(A, lambda v: oracle.solve(Fo, v), p.rhs[:, k], tol=TOL, restart=30, maxit=500)
    ro = np.linalg.norm(A @ o["x"] - p.rhs[:, k]) / np.linalg.norm(p.rhs[:, k])
    bound = _smin_bound(A, p.rhs[:, k], resm[k], ro)
    d = np.linalg.norm(xm[:, k] - o["x"])
    print(f"[c2] mixed vs FP64 oracle FGMRES: {d / np.linalg.norm(o['x']):.2e} relative "
          f"(bound {bound / np.linalg.norm(o['x']):.2e}); iterations mixed {int(itm[k])}, FP64 {int(its[k])}, "
          f"oracle {o['iters']}", flush=True)
    assert d <= 1.01 * bound
    assert abs(int(its[k]) - o["iters"]) <= 1


def test_convdiff3d_large_block_shape(lx):
    csr, n, perm, lp, depth, rng = grid("convdiff3d", 32, 128, 3)
    eps = 1e-3
    print(f"[c3-shape] n={n} depth={depth}", flush=True)
    F = lx.Factor(*csr, perm, lp, depth, eps)
    Fo = oracle_matching(F, csr, perm, lp, depth, eps)
    wide = sum(1 for c in Fo.compressions if c.m > 192 or c.rows * c.m >= 1e6)
    tall = sum(1 for c in Fo.compressions if 64 < c.m <= 192 and 3e5 <= c.rows * c.m < 1e6)
    print(f"[c3-shape] split-path blocks {wide}, panel tall-QR blocks {tall}", flush=True)
    assert wide >= 8 and tall >= 5
    b = rng.uniform(-1, 1, (n, 2))
    x = F.solve(b)
    xo = np.column_stack([oracle.solve(Fo, b[:, k]) for k in range(2)])
    err = relerr(x, xo)
    print(f"[c3-shape] FP64 solve vs oracle: {err:.2e}", flush=True)
    assert err <= TOL
    A = sp.csr_matrix((csr[2], csr[1], csr[0]), shape=(n, n))
    Fm = lx.Factor(*csr, perm, lp, depth, eps, precision="mixed")
    xm, itm, rm = Fm.gmres(b, tol=TOL, restart=30, maxit=500)
    resm = np.linalg.norm(A @ xm - b, axis=0) / np.linalg.norm(b, axis=0)
    assert (resm <= TOL).all()
    # mixed answer against the oracle-preconditioned FP64 answer
    o = oracle.fgmres(A, lambda v: oracle.solve(Fo, v), b[:, 0], tol=TOL, restart=30, maxit=500)
    ro = np.linalg.norm(A @ o["x"] - b[:, 0]) / np.linalg.norm(b[:, 0])
    bound = _smin_bound(A, b[:, 0], resm[0], ro)
    d = np.linalg.norm(xm[:, 0] - o["x"])
    print(f"[c3-shape] mixed vs FP64 oracle FGMRES: {d / np.linalg.norm(o['x']):.2e} relative "
          f"(bound {bound / np.linalg.norm(o['x']):.2e}), iterations {int(itm[0])} vs {o['iters']}", flush=True)
    assert d <= 1.01 * bound


def test_batched_factor_against_oracle(lx):
    ins = [grid("lognormal2d", 40, 32, 1), grid("lognormal3d", 12, 32, 2), grid("convdiff2d", 64, 64, 3)]
    eps = 1e-4
    Fs = lx.factor_batch([(*csr, perm, lp, depth) for csr, n, perm, lp, depth, _ in ins], eps)
    for i in (0, 1, 2):
        csr, n, perm, lp, depth, rng = ins[i]
        Fo = oracle_matching(Fs[i], csr, perm, lp, depth, eps)
        b = rng.uniform(-1, 1, (n, 2))
        x = Fs[i].solve(b)
        xo = np.column_stack([oracle.solve(Fo, b[:, k]) for k in range(2)])
        err = relerr(x, xo)
        print(f"[batch] system {i}: solve vs oracle {err:.2e}", flush=True)
        assert err <= TOL
    # batched solve of all three against the oracle
    import torch
    nrhs = 2
    bs, xs, ref = [], [], []
    for i, (csr, n, perm, lp, depth, rng) in enumerate(ins):
        b = rng.uniform(-1, 1, (n, nrhs))
        bs.append(torch.from_numpy(np.ascontiguousarray(b.T)).to("cuda:0"))
        xs.append(torch.zeros_like(bs[-1]))
        ref.append(b)
    lx.solve_batch_dev(Fs, nrhs, [b.data_ptr() for b in bs], [x.data_ptr() for x in xs])
    for i, (csr, n, perm, lp, depth, rng) in enumerate(ins):
        Fo = oracle_matching(Fs[i], csr, perm, lp, depth, eps)
        xo = np.column_stack([oracle.solve(Fo, ref[i][:, k]) for k in range(nrhs)])
        err = relerr(xs[i].cpu().numpy().T, xo)
        assert err <= TOL, (i, err)
    its_b, rr_b, st = lx.gmres_batch_dev(Fs, nrhs, [b.data_ptr() for b in bs], [x.data_ptr() for x in xs],
                                         tol=TOL, restart=30, maxit=500)
    for i, (csr, n, perm, lp, depth, rng) in enumerate(ins):
        A = sp.csr_matrix((csr[2], csr[1], csr[0]), shape=(n, n))
        Fo = oracle_matching(Fs[i], csr, perm, lp, depth, eps)
        X = xs[i].cpu().numpy().T
        for k in range(nrhs):
            res = np.linalg.norm(A @ X[:, k] - ref[i][:, k]) / np.linalg.norm(ref[i][:, k])
            o = oracle.fgmres(A, lambda v: oracle.solve(Fo, v), ref[i][:, k], tol=TOL, restart=30, maxit=500)
            assert res <= TOL
            assert abs(int(its_b[i, k]) - o["iters"]) <= 1, (i, k, its_b[i, k], o["iters"])


@pytest.mark.parametrize("cycle", [None, 2])
def test_served_answers_against_oracle(lx, cycle):
    """Served solves (continuous batching across resident handles; with cycle,
    rounds of one FGMRES(2) cycle that continue unconverged right-hand sides
    from their iterate) reach the tolerance, and each equals the
    oracle-preconditioned FP64 FGMRES answer within the conditioning bound."""
    from paper_1510_07363_amd.serve import LoraxBackend, Server, SystemSpec
    ins = {"a": (grid("lognormal2d", 48, 16, 11), 1e-5), "b": (grid("lognormal3d", 12, 32, 12), 1e-3)}
    for precision in ("fp64", "mixed"):
        srv = Server(LoraxBackend(precision=precision), 8 << 30, tol=TOL, cycle=cycle)
        for key, ((csr, n, perm, lp, depth, rng), eps) in ins.items():
            srv.register(SystemSpec(key, csr[0], csr[1], csr[2], perm, lp, depth, eps))
        rng = np.random.default_rng(99)
        reqs = [("a", rng.uniform(-1, 1, (ins["a"][0][1], 2))), ("b", rng.uniform(-1, 1, (ins["b"][0][1], 3))),
                ("a", rng.uniform(-1, 1, (ins["a"][0][1], 1)))]
        futs = [srv.submit(k, b) for k, b in reqs]
        srv.run_until_idle()
        for (key, b), f in zip(reqs, futs):
            (csr, n, perm, lp, depth, _), eps = ins[key]
            A = sp.csr_matrix((csr[2], csr[1], csr[0]), shape=(n, n))
            Fo = oracle.factor(*csr, perm, lp, depth, eps, check=False)
            x, its, rr = f.result()
            for k in range(b.shape[1]):
                r = np.linalg.norm(A @ x[:, k] - b[:, k]) / np.linalg.norm(b[:, k])
                o = oracle.fgmres(A, lambda v: oracle.solve(Fo, v), b[:, k], tol=TOL, restart=30, maxit=500)
                ro = np.linalg.norm(A @ o["x"] - b[:, k]) / np.linalg.norm(b[:, k])
                smin = np.linalg.svd(A.toarray(), compute_uv=False)[-1]
                bound = (r + ro) * np.linalg.norm(b[:, k]) / smin
                assert r <= TOL
                assert np.linalg.norm(x[:, k] - o["x"]) <= 1.01 * bound + 1e-14, (precision, key, k)
        if cycle:
            assert srv.n_rounds >= 2
        srv.close()


def test_gmres_from_initial_guess(lx):
    """lrx_gmres_batch_dev_x0: a converged iterate stops at once; a cycle-limited
    first call (ENOCONV) continued from its iterate reaches the tolerance; a
    zero right-hand side returns x = 0 whatever the guess."""
    import torch
    csr, n, perm, lp, depth, rng = grid("varcoef2d", 48, 16, 21)
    A = sp.csr_matrix((csr[2], csr[1], csr[0]), shape=(n, n))
    F = lx.Factor(*csr, perm, lp, depth, 1e-1)
    B = rng.uniform(-1, 1, (n, 3))
    B[:, 2] = 0.0
    b = torch.from_numpy(np.ascontiguousarray(B.T)).to("cuda:0")
    x = torch.zeros_like(b)
    its1, rr1, st1 = lx.gmres_batch_dev([F], 3, [b.data_ptr()], [x.data_ptr()], tol=TOL, restart=2, maxit=2)
    assert st1 == lx.LRX_ENOCONV and rr1[0, 0] > TOL
    x[2].fill_(7.0)                                   # guess for the zero right-hand side
    its2, rr2, st2 = lx.gmres_batch_dev([F], 3, [b.data_ptr()], [x.data_ptr()], tol=TOL, restart=2, maxit=200,
                                        x0=True)
    assert st2 == lx.LRX_OK
    X = x.cpu().numpy().T
    r = np.linalg.norm(A @ X[:, :2] - B[:, :2], axis=0) / np.linalg.norm(B[:, :2], axis=0)
    assert (r <= TOL).all() and (rr2[0, :2] <= TOL).all()
    assert np.all(X[:, 2] == 0.0)
    its3, rr3, st3 = lx.gmres_batch_dev([F], 3, [b.data_ptr()], [x.data_ptr()], tol=TOL, restart=2, maxit=200,
                                        x0=True)
    assert st3 == lx.LRX_OK and (its3 == 0).all()
