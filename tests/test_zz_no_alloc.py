"""The allocation-free solve entry point (lrx_solve_dev_noalloc) against
lrx_solve_dev through the C ABI: two calls in a row on the library's static
device scratch, the second with a smaller input (another handle, fewer
right-hand sides), each equal to lrx_solve_dev's result bit for bit; sizes
beyond the scratch are rejected on the host."""
import ctypes

import numpy as np
import pytest

from paper_1510_07363_amd import workloads as w

pytestmark = pytest.mark.gpu


def _system(nx, leaf, seed):
    rng = np.random.default_rng(seed)
    csr = w.diffusion2d(np.exp(rng.standard_normal(nx * nx)), (nx, nx))
    n = nx * nx
    depth = w.tree_depth(n, leaf)
    perm, lp = w.rcb_tree(w.grid_coords((nx, nx)), depth)
    return csr, n, perm, lp, depth, rng


def test_noalloc_solve_equals_solve_dev():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    torch.cuda.set_device(0)
    from paper_1510_07363_amd import lorax as lx
    big = _system(64, 32, 1)
    small = _system(24, 16, 2)
    Fb = lx.Factor(*big[0], big[2], big[3], big[4], 1e-4)
    Fs = lx.Factor(*small[0], small[2], small[3], small[4], 1e-4, precision="mixed")
    for F, (csr, n, perm, lp, depth, rng), nrhs in ((Fb, big, 6), (Fs, small, 2)):
        b = torch.from_numpy(rng.uniform(-1, 1, (nrhs, n))).to("cuda:0")      # n x nrhs column-major
        x_ref = torch.zeros_like(b)
        x_na = torch.full_like(b, float("nan"))
        F.solve_dev(b.data_ptr(), x_ref.data_ptr(), nrhs)
        st = lx._lib.lrx_solve_dev_noalloc(F._h, nrhs, ctypes.c_void_p(b.data_ptr()),
                                           ctypes.c_void_p(x_na.data_ptr()))
        assert st == lx.LRX_OK, lx._lib.lrx_last_error().decode()
        torch.cuda.synchronize()
        assert torch.equal(x_na, x_ref), float((x_na - x_ref).abs().max())
    # more right-hand sides than the scratch holds: rejected before any launch
    wide = _system(136, 64, 3)
    Fw = lx.Factor(*wide[0], wide[2], wide[3], wide[4], 1e-4)
    n_ext = Fw.stats()["extended_size"]
    too_many = (32 << 20) // (8 * n_ext) + 1
    assert too_many <= 256
    b = torch.zeros((too_many, wide[1]), dtype=torch.float64, device="cuda:0")
    x = torch.zeros_like(b)
    st = lx._lib.lrx_solve_dev_noalloc(Fw._h, too_many, ctypes.c_void_p(b.data_ptr()), ctypes.c_void_p(x.data_ptr()))
    assert st == lx.LRX_EINVAL and "scratch" in lx._lib.lrx_last_error().decode()
    assert torch.count_nonzero(x) == 0
