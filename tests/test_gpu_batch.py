"""Batched solves across factorizations (lrx_solve_batch_dev) on the GPU.

Several factorizations of different sizes, kinds and depths are solved in one
call: every (level, colour) step of the sweeps is a single launch over the
nodes of all of them.  Each result must equal the solve of that factorization
alone (same kernels, same per-node programs: bit for bit), in FP64, in mixed
precision and with both precisions in one batch; a handle that appears twice
is rejected.
"""
import numpy as np
import pytest
import scipy.sparse as sp

from paper_1510_07363_amd import workloads as w

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def env():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    torch.cuda.set_device(0)
    from paper_1510_07363_amd import lorax
    return lorax, torch


def _system(kind, nx, leaf, seed):
    rng = np.random.default_rng(seed)
    if kind == "diff2d":
        csr = w.diffusion2d(np.exp(rng.standard_normal(nx * nx)), (nx, nx))
        co = w.grid_coords((nx, nx))
    elif kind == "diff3d":
        csr = w.diffusion3d(np.exp(rng.standard_normal(nx ** 3)), (nx, nx, nx))
        co = w.grid_coords((nx, nx, nx))
    elif kind == "convdiff2d":
        csr, co = w.convdiff2d(nx), w.grid_coords((nx, nx))
    else:
        raise KeyError(kind)
    n = len(csr[0]) - 1
    depth = w.tree_depth(n, leaf)
    perm, lp = w.rcb_tree(co, depth)
    return csr, n, perm, lp, depth, rng


SYSTEMS = [("diff2d", 40, 32, 1), ("diff3d", 12, 32, 2), ("convdiff2d", 64, 64, 3), ("diff2d", 24, 16, 4)]


@pytest.mark.parametrize("precision", ["fp64", "mixed", "both"])
def test_batch_equals_single_solves(env, precision):
    lx, torch = env
    nrhs = 4
    facs, bs, xs, ref = [], [], [], []
    for i, (kind, nx, leaf, seed) in enumerate(SYSTEMS):
        csr, n, perm, lp, depth, rng = _system(kind, nx, leaf, seed)
        prec = precision if precision != "both" else ("fp64", "mixed")[i % 2]
        F = lx.Factor(*csr, perm, lp, depth, 1e-4, precision=prec)
        b = torch.from_numpy(np.asfortranarray(rng.uniform(-1, 1, (n, nrhs))).T.copy()).to("cuda:0")
        x1 = torch.zeros_like(b)
        F.solve_dev(b.data_ptr(), x1.data_ptr(), nrhs)
        facs.append(F)
        bs.append(b)
        xs.append(torch.zeros_like(b))
        ref.append(x1)
    torch.cuda.synchronize()
    lx.solve_batch_dev(facs, nrhs, [b.data_ptr() for b in bs], [x.data_ptr() for x in xs])
    for x, r in zip(xs, ref):
        assert torch.equal(x, r), float((x - r).abs().max())


def test_batch_rejects_repeated_handle(env):
    lx, torch = env
    csr, n, perm, lp, depth, rng = _system("diff2d", 24, 16, 7)
    Fa = lx.Factor(*csr, perm, lp, depth, 1e-4)
    b = torch.zeros((1, n), dtype=torch.float64, device="cuda:0")
    x = torch.zeros_like(b)
    y = torch.zeros_like(b)
    with pytest.raises(lx.LoraxError) as e:
        lx.solve_batch_dev([Fa, Fa], 1, [b.data_ptr()] * 2, [x.data_ptr(), y.data_ptr()])
    assert e.value.status == lx.LRX_EINVAL


def _batch_inputs(systems):
    out = []
    for kind, nx, leaf, seed in systems:
        csr, n, perm, lp, depth, rng = _system(kind, nx, leaf, seed)
        out.append((csr, n, perm, lp, depth, rng))
    return out


# sizes and kinds vary so the systems have different depths, colour counts and
# ranks; the 3D system with 128-point leaves has compressions with c > 64
FSYSTEMS = [("diff2d", 40, 32, 11), ("diff3d", 12, 32, 12), ("convdiff2d", 64, 64, 13),
            ("diff2d", 24, 16, 14), ("diff3d", 16, 128, 15)]


@pytest.mark.parametrize("precision,compress", [("fp64", "svd"), ("mixed", "svd"), ("fp64", "rrqr")])
def test_factor_batch_equals_single_factors(env, precision, compress):
    """Each factorization of a batch equals the same system factored alone: the
    same ranks, truncation tails and storage, and bit-identical solves."""
    lx, torch = env
    ins = _batch_inputs(FSYSTEMS)
    eps = 1e-4
    batch = lx.factor_batch([(*csr, perm, lp, depth) for csr, n, perm, lp, depth, _ in ins], eps,
                            compress=compress, precision=precision)
    assert len(batch) == len(ins)
    nrhs = 3
    for i, ((csr, n, perm, lp, depth, rng), Fb) in enumerate(zip(ins, batch)):
        Fs = lx.Factor(*csr, perm, lp, depth, eps, compress=compress, precision=precision)
        rs, rb = Fs.ranks(), Fb.ranks()
        for a, b in zip(rs, rb):
            assert np.array_equal(a, b), i
        Ss, Sb = Fs.stats(), Fb.stats()
        for key in ("factor_bytes", "solve_bytes", "extended_size", "n_compressions", "factor_flops"):
            assert Ss[key] == Sb[key], (i, key, Ss[key], Sb[key])
        assert Ss["max_compression_error"] == Sb["max_compression_error"]
        b = torch.from_numpy(rng.uniform(-1, 1, (nrhs, n))).to("cuda:0")
        xs, xb = torch.zeros_like(b), torch.zeros_like(b)
        Fs.solve_dev(b.data_ptr(), xs.data_ptr(), nrhs)
        Fb.solve_dev(b.data_ptr(), xb.data_ptr(), nrhs)
        torch.cuda.synchronize()
        assert torch.equal(xs, xb), (i, float((xs - xb).abs().max()))
        # and the batched factor is a working preconditioner of its own system
        x, its, rr = Fb.gmres(rng.uniform(-1, 1, n), tol=1e-10)
        assert rr[0] <= 1e-10


def test_factor_batch_single_system_and_errors(env):
    lx, torch = env
    (csr, n, perm, lp, depth, rng), = _batch_inputs([("diff2d", 24, 16, 21)])
    Fb, = lx.factor_batch([(*csr, perm, lp, depth)], 1e-6)
    Fs = lx.Factor(*csr, perm, lp, depth, 1e-6)
    b = rng.uniform(-1, 1, n)
    assert np.array_equal(Fb.solve(b), Fs.solve(b))
    # a bad tree in one system fails the whole batch and names that system
    bad_lp = lp.copy()
    bad_lp[-1] += 1
    with pytest.raises(lx.LoraxError) as e:
        lx.factor_batch([(*csr, perm, lp, depth), (*csr, perm, bad_lp, depth)], 1e-6)
    assert e.value.status == lx.LRX_EINVAL and "system 1" in str(e.value)
    # an exactly singular pivot in one system: LRX_ESINGULAR for the batch

    A = sp.csr_matrix((csr[2], csr[1], csr[0]), shape=(n, n)).tolil()
    for r in perm[lp[0]:lp[1]]:
        A[r, :] = 0.0
        A[:, r] = 0.0
    A = A.tocsr()
    A.sort_indices()
    A.eliminate_zeros()
    sing = (A.indptr.astype(np.int64), A.indices.astype(np.int32), A.data, perm, lp, depth)
    with pytest.raises(lx.LoraxError) as e:
        lx.factor_batch([(*csr, perm, lp, depth), sing], 1e-6)
    assert e.value.status == lx.LRX_ESINGULAR and "system 1" in str(e.value)
    # the library still works after the failed batches
    F2, = lx.factor_batch([(*csr, perm, lp, depth)], 1e-6)
    assert np.array_equal(F2.solve(b), Fs.solve(b))


def test_gmres_batch_equals_single_gmres(env):
    """FGMRES of several systems in lock-step (lrx_gmres_batch_dev): each system's
    iterates are computed by the same launches over its own rows as when it runs
    alone, so x, iteration counts and residuals are bit-identical to
    lrx_gmres_dev; systems of different sizes converge at different steps and
    drop out; a zero right-hand side stops at once with x = 0."""
    lx, torch = env
    nrhs = 3
    ins = _batch_inputs(FSYSTEMS)
    facs = lx.factor_batch([(*csr, perm, lp, depth) for csr, n, perm, lp, depth, _ in ins], 1e-3,
                           precision="mixed")
    bs, xs = [], []
    for i, (csr, n, perm, lp, depth, rng) in enumerate(ins):
        b = rng.uniform(-1, 1, (nrhs, n))
        if i == 1:
            b[2] = 0.0
        bs.append(torch.from_numpy(b).to("cuda:0"))
        xs.append(torch.zeros_like(bs[-1]))
    its, rr, st = lx.gmres_batch_dev(facs, nrhs, [b.data_ptr() for b in bs], [x.data_ptr() for x in xs],
                                     tol=1e-10)
    assert st == lx.LRX_OK
    for i, ((csr, n, perm, lp, depth, rng), F) in enumerate(zip(ins, facs)):
        x1 = torch.zeros_like(bs[i])
        its1, rr1, st1 = F.gmres_dev(bs[i].data_ptr(), x1.data_ptr(), nrhs, tol=1e-10)
        assert st1 == lx.LRX_OK
        assert np.array_equal(its[i], its1) and np.array_equal(rr[i], rr1), (i, its[i], its1)
        assert torch.equal(xs[i], x1), (i, float((xs[i] - x1).abs().max()))
        A = sp.csr_matrix((csr[2], csr[1], csr[0]), shape=(n, n))
        X = xs[i].cpu().numpy()
        B = bs[i].cpu().numpy()
        for k in range(nrhs):
            nb = np.linalg.norm(B[k])
            if nb == 0:
                assert its[i][k] == 0 and not X[k].any()
                continue
            assert np.linalg.norm(A @ X[k] - B[k]) / nb <= 1e-10


def test_gmres_batch_nonconvergence_and_errors(env):
    lx, torch = env
    ins = _batch_inputs([("diff2d", 24, 16, 31), ("diff2d", 32, 16, 32)])
    facs = [lx.Factor(*csr, perm, lp, depth, 0.5) for csr, n, perm, lp, depth, _ in ins]
    bs = [torch.from_numpy(rng.uniform(-1, 1, (1, n))).to("cuda:0") for csr, n, perm, lp, depth, rng in ins]
    xs = [torch.zeros_like(b) for b in bs]
    its, rr, st = lx.gmres_batch_dev(facs, 1, [b.data_ptr() for b in bs], [x.data_ptr() for x in xs],
                                     tol=1e-14, restart=2, maxit=3)
    assert st == lx.LRX_ENOCONV and (its == 3).all() and (rr > 1e-14).all()
    with pytest.raises(lx.LoraxError) as e:
        lx.gmres_batch_dev([facs[0], facs[0]], 1, [bs[0].data_ptr()] * 2, [xs[0].data_ptr(), xs[1].data_ptr()])
    assert e.value.status == lx.LRX_EINVAL
