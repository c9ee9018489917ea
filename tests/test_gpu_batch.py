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
