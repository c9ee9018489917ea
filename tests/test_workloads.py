"""Structure checks of the seeded synthetic inputs (sizes, patterns, cluster tree)."""
import numpy as np
import pytest
import scipy.sparse as sp

from paper_1510_07363_amd import workloads as w


def test_poisson32():
    p = w.make_config("poisson2d_32")
    assert (p.n, p.nnz, p.depth) == (1024, 4992, 6)
    A = p.scipy()
    assert abs(A - A.T).max() == 0
    assert np.allclose(A.diagonal(), 4.0)
    box = p.coords[p.perm[p.leaf_ptr[0]:p.leaf_ptr[1]]]
    assert tuple(box.max(0) - box.min(0) + 1) == (4, 4)


def test_varcoef256_structure():
    p = w.make_config("varcoef2d_256")
    assert (p.n, p.nnz, p.depth) == (65536, 326656, 10)
    assert p.rhs.shape == (65536, 8)
    A = p.scipy()
    assert abs(A - A.T).max() == 0
    # M-matrix with strictly positive row sums only on the boundary (Dirichlet)
    off = A - sp.diags(A.diagonal())
    assert off.max() <= 0
    rs = np.asarray(A.sum(axis=1)).ravel()
    assert rs.min() >= -1e-12
    box = p.coords[p.perm[p.leaf_ptr[5]:p.leaf_ptr[6]]]
    assert tuple(box.max(0) - box.min(0) + 1) == (8, 8)


def test_convdiff64_structure():
    csr = w.convdiff3d(64)
    n = 64 ** 3
    assert int(csr[0][-1]) == 1810432
    depth = w.tree_depth(n, 128)
    assert depth == 11


def test_convdiff_small_stencil():
    csr = w.convdiff3d(4)
    A = sp.csr_matrix((csr[2], csr[1], csr[0]), shape=(64, 64)).toarray()
    h = 1.0 / 5
    # centre cell (1,1,1) -> index 1 + 4 + 16
    c = 21
    assert A[c, c] == pytest.approx(6 + h * 17.5)
    assert A[c, c + 1] == -1 and A[c, c + 4] == -1 and A[c, c + 16] == -1
    assert A[c, c - 1] == pytest.approx(-1 - h * 10)
    assert A[c, c - 4] == pytest.approx(-1 - h * 5)
    assert A[c, c - 16] == pytest.approx(-1 - h * 2.5)


def test_rcb_is_nested_and_balanced():
    co = w.grid_coords((12, 10))
    perm, lp = w.rcb_tree(co, 4)
    assert sorted(perm.tolist()) == list(range(120))
    sizes = np.diff(lp)
    assert sizes.min() >= 7 and sizes.max() <= 8


def test_gaussian_field_stats():
    g = w.gaussian_field_2d((128, 128), np.random.default_rng(0), 8.0)
    assert abs(g.mean()) < 1e-12 and abs(g.std() - 1) < 1e-12
    G = g.reshape(128, 128)
    # neighbour correlation of exp(-r^2/(2*64)) at r=1 ~ 0.992
    c1 = np.mean(G[:, 1:] * G[:, :-1])
    assert 0.95 < c1 < 1.0
