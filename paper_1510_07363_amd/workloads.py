"""Seeded synthetic workloads: sparse matrices, cluster trees and right-hand sides.

This module only *builds inputs*.  It holds none of the solver's arithmetic, so
both the CPU oracle (test infrastructure) and the HIP path read what it makes.

Matrices are PDE stencils of the shapes the paper benchmarks on (Sec. 6: Poisson
on structured grids, variable-coefficient diffusion, convection-diffusion), all
scaled by h^2 (unscaled stencil weights), in CSR with int64 row pointers, int32
column indices, sorted columns and no duplicates.  Grid ordering is x-fastest.

The cluster tree is a recursive coordinate bisection (RCB) giving the nested,
binary partitionings P_0..P_l of Sec. 3 (Def. "nested partitionings"): every
cluster at level i is the union of its two children at level i+1, so the leaf
clusters are contiguous ranges of a permutation.
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field

import numpy as np
import scipy.sparse as sp

__all__ = [
    "Problem", "poisson2d", "diffusion2d", "diffusion3d", "convdiff2d", "convdiff3d",
    "gaussian_field_2d", "rcb_tree", "tree_depth", "uniform_rhs", "grid_coords",
    "make_config", "CONFIGS", "make_batch", "make_serve_stream", "build_serve_system",
]


# ----------------------------------------------------------------------------- data
@dataclass
class Problem:
    """One linear system A x = b with its cluster tree."""
    name: str
    n: int
    row_ptr: np.ndarray          # int64[n+1]
    col_idx: np.ndarray          # int32[nnz]
    val: np.ndarray              # float64[nnz]
    coords: np.ndarray           # float64[n, dim]
    perm: np.ndarray             # int32[n]  tree position -> original row
    leaf_ptr: np.ndarray         # int32[2^depth + 1]
    depth: int
    epsilon: float
    rhs: np.ndarray              # float64[n, nrhs] (column-major use: rhs[:, k])
    meta: dict = field(default_factory=dict)

    @property
    def nnz(self) -> int:
        return int(self.row_ptr[-1])

    def scipy(self) -> sp.csr_matrix:
        return sp.csr_matrix((self.val, self.col_idx, self.row_ptr), shape=(self.n, self.n))


def _to_csr(rows, cols, vals, n):
    m = sp.coo_matrix((vals, (rows, cols)), shape=(n, n)).tocsr()
    m.sum_duplicates()
    m.sort_indices()
    return (m.indptr.astype(np.int64), m.indices.astype(np.int32), m.data.astype(np.float64))


def grid_coords(shape):
    """Integer grid coordinates, x fastest: index = ix + nx*iy (+ nx*ny*iz)."""
    axes = [np.arange(s, dtype=np.float64) for s in shape]
    mesh = np.meshgrid(*axes, indexing="ij")          # mesh[d][ix, iy, ...]
    # flatten with x fastest -> transpose so that the last flattened axis is x
    cols = [m.transpose(tuple(range(len(shape)))[::-1]).ravel() for m in mesh]
    return np.stack(cols, axis=1)


# ----------------------------------------------------------------- stencil assembly
def _assemble(shape, plus_coef, minus_coef, diag):
    """Generic assembly: A[c,c] = diag[c]; A[c, c+e_d] = -plus_coef[d][c];
    A[c, c-e_d] = -minus_coef[d][c] (entries that fall outside are dropped)."""
    dims = len(shape)
    n = int(np.prod(shape))
    strides = [1]
    for s in shape[:-1]:
        strides.append(strides[-1] * s)
    idx = np.arange(n).reshape(tuple(shape[::-1]))     # idx[iz, iy, ix]
    rows = [np.arange(n)]
    cols = [np.arange(n)]
    vals = [diag.ravel()]
    for d in range(dims):
        ax = dims - 1 - d                               # numpy axis of grid axis d
        sl_lo = [slice(None)] * dims
        sl_hi = [slice(None)] * dims
        sl_lo[ax] = slice(0, shape[d] - 1)
        sl_hi[ax] = slice(1, shape[d])
        a = idx[tuple(sl_lo)].ravel()                   # cell c with a +d neighbour
        b = idx[tuple(sl_hi)].ravel()                   # that neighbour
        pc = plus_coef[d].reshape(tuple(shape[::-1]))[tuple(sl_lo)].ravel()
        mc = minus_coef[d].reshape(tuple(shape[::-1]))[tuple(sl_hi)].ravel()
        rows += [a, b]
        cols += [b, a]
        vals += [-pc, -mc]
    r = np.concatenate(rows)
    c = np.concatenate(cols)
    v = np.concatenate(vals)
    return _to_csr(r, c, v, n)


def poisson2d(nx, ny=None):
    """-Laplace, 5-point, Dirichlet: diagonal 4, off-diagonals -1 (scaled by h^2)."""
    ny = nx if ny is None else ny
    shape = (nx, ny)
    n = nx * ny
    one = np.ones(n)
    return _assemble(shape, [one, one], [one, one], 4.0 * one)


def _harmonic_faces(kappa_grid, shape):
    """Face coefficients (harmonic mean of the two cells) and diagonal, Dirichlet
    boundary faces using the cell's own coefficient."""
    dims = len(shape)
    kap = kappa_grid.reshape(tuple(shape[::-1]))
    diag = np.zeros_like(kap)
    plus = []
    for d in range(dims):
        ax = dims - 1 - d
        lo = [slice(None)] * dims
        hi = [slice(None)] * dims
        lo[ax] = slice(0, shape[d] - 1)
        hi[ax] = slice(1, shape[d])
        ka = kap[tuple(lo)]
        kb = kap[tuple(hi)]
        face = 2.0 * ka * kb / (ka + kb)
        full = np.zeros_like(kap)
        full[tuple(lo)] = face
        plus.append(full.ravel())
        diag[tuple(lo)] += face
        diag[tuple(hi)] += face
        first = [slice(None)] * dims
        last = [slice(None)] * dims
        first[ax] = slice(0, 1)
        last[ax] = slice(shape[d] - 1, shape[d])
        diag[tuple(first)] += kap[tuple(first)]
        diag[tuple(last)] += kap[tuple(last)]
    # minus coefficient at cell c+e_d equals the plus coefficient at c
    minus = []
    for d in range(dims):
        ax = dims - 1 - d
        p = plus[d].reshape(kap.shape)
        m = np.zeros_like(kap)
        lo = [slice(None)] * dims
        hi = [slice(None)] * dims
        lo[ax] = slice(0, shape[d] - 1)
        hi[ax] = slice(1, shape[d])
        m[tuple(hi)] = p[tuple(lo)]
        minus.append(m.ravel())
    return plus, minus, diag.ravel()


def diffusion2d(kappa, shape):
    """-div(kappa grad u), cell-centred, 5-point, harmonic face means (SPD)."""
    plus, minus, diag = _harmonic_faces(np.asarray(kappa, dtype=np.float64).ravel(), shape)
    return _assemble(shape, plus, minus, diag)


def diffusion3d(kappa, shape):
    """-div(kappa grad u), cell-centred, 7-point, harmonic face means (SPD)."""
    plus, minus, diag = _harmonic_faces(np.asarray(kappa, dtype=np.float64).ravel(), shape)
    return _assemble(shape, plus, minus, diag)


def _convdiff(shape, w, h):
    """-Laplace u + w.grad u, first-order upwind (w > 0: backward differences),
    scaled by h^2: diagonal 2*dim + h*sum(w); -1 on +d; -1 - h*w_d on -d."""
    n = int(np.prod(shape))
    one = np.ones(n)
    dims = len(shape)
    plus = [one.copy() for _ in range(dims)]
    minus = [(1.0 + h * w[d]) * one for d in range(dims)]
    diag = (2.0 * dims + h * float(np.sum(w))) * one
    return _assemble(shape, plus, minus, diag)


def convdiff3d(nx, pe=10.0, direction=(1.0, 0.5, 0.25)):
    h = 1.0 / (nx + 1)
    w = np.asarray(direction, dtype=np.float64) * pe
    return _convdiff((nx, nx, nx), w, h)


def convdiff2d(nx, pe=10.0, direction=(1.0, 0.5)):
    h = 1.0 / (nx + 1)
    w = np.asarray(direction, dtype=np.float64) * pe
    return _convdiff((nx, nx), w, h)


def gaussian_field_2d(shape, rng, corr_len=8.0):
    """Stationary Gaussian field: white noise N(0,1) convolved periodically (FFT)
    with a Gaussian of std corr_len/sqrt(2) cells, so the covariance is
    proportional to exp(-r^2 / (2 corr_len^2)); standardised to mean 0, std 1."""
    nx, ny = shape
    wn = rng.standard_normal((ny, nx))
    s = corr_len / math.sqrt(2.0)
    dx = np.minimum(np.arange(nx), nx - np.arange(nx)).astype(np.float64)
    dy = np.minimum(np.arange(ny), ny - np.arange(ny)).astype(np.float64)
    ker = np.exp(-(dy[:, None] ** 2 + dx[None, :] ** 2) / (2.0 * s * s))
    g = np.fft.ifft2(np.fft.fft2(wn) * np.fft.fft2(ker)).real
    g = (g - g.mean()) / g.std()
    return g.ravel()                                   # x fastest


# ------------------------------------------------------------------------ cluster tree
def tree_depth(n, leaf_size):
    """Depth l = ceil(log2(n / leaf)) so that n_{P_i} = 2^i (Def. nested partitionings)."""
    return max(0, int(math.ceil(math.log2(n / float(leaf_size)) - 1e-12)))


def rcb_tree(coords, depth):
    """Recursive coordinate bisection to `depth` levels.

    Each cluster is split on the axis of largest coordinate extent (ties: x, then
    y, then z); points are sorted by (coordinate, original index) and the first
    floor(|C|/2) go to child 0 (cluster 2c at the next level).  Returns
    (perm[int32 n], leaf_ptr[int32 2^depth+1])."""
    coords = np.asarray(coords, dtype=np.float64)
    n = coords.shape[0]
    if n < (1 << depth):
        raise ValueError("fewer points than leaves")
    clusters = [np.arange(n)]
    for _ in range(depth):
        nxt = []
        for idx in clusters:
            pts = coords[idx]
            ext = pts.max(axis=0) - pts.min(axis=0)
            ax = int(np.argmax(ext))
            order = np.lexsort((idx, pts[:, ax]))
            srt = idx[order]
            h = len(srt) // 2
            nxt.append(srt[:h])
            nxt.append(srt[h:])
        clusters = nxt
    perm = np.concatenate(clusters).astype(np.int32)
    leaf_ptr = np.zeros(len(clusters) + 1, dtype=np.int32)
    leaf_ptr[1:] = np.cumsum([len(c) for c in clusters])
    return perm, leaf_ptr


def uniform_rhs(n, nrhs, rng):
    """Right-hand sides with entries uniform in [-1, 1]; shape (n, nrhs)."""
    return rng.uniform(-1.0, 1.0, size=(nrhs, n)).T.copy()


# ------------------------------------------------------------------------- configs
def _finish(name, csr, coords, leaf, eps, nrhs, rng, meta):
    row_ptr, col_idx, val = csr
    n = len(row_ptr) - 1
    depth = tree_depth(n, leaf)
    perm, leaf_ptr = rcb_tree(coords, depth)
    b = uniform_rhs(n, nrhs, rng)
    meta = dict(meta, leaf=leaf)
    return Problem(name, n, row_ptr, col_idx, val, coords, perm, leaf_ptr, depth, eps, b, meta)


def make_config(which, seed=None, size=None):
    """Build one of the named workloads.

    poisson2d_32      : 2-D 5-point Poisson 32x32 (n=1,024), leaf 16, eps 1e-12, 1 RHS
    varcoef2d_256     : 2-D diffusion 256x256 (n=65,536), kappa=exp(g), g Gaussian
                        (sigma 1, correlation length 8), leaf 64, eps 1e-4, 8 RHS
    convdiff3d_64     : 3-D upwind convection-diffusion 64^3 (n=262,144), w=(1,.5,.25)*10,
                        leaf 128, eps 1e-3, 8 RHS
    `size` overrides the grid side (same recipe, smaller grid) for quick tests.
    """
    if which == "poisson2d_32":
        seed = 1 if seed is None else seed
        nx = size or 32
        rng = np.random.default_rng(seed)
        csr = poisson2d(nx)
        return _finish(which, csr, grid_coords((nx, nx)), 16, 1e-12, 1, rng,
                       {"grid": (nx, nx), "seed": seed})
    if which == "varcoef2d_256":
        seed = 2 if seed is None else seed
        nx = size or 256
        rng = np.random.default_rng(seed)
        g = gaussian_field_2d((nx, nx), rng, 8.0)
        kappa = np.exp(g)
        csr = diffusion2d(kappa, (nx, nx))
        return _finish(which, csr, grid_coords((nx, nx)), 64, 1e-4, 8, rng,
                       {"grid": (nx, nx), "seed": seed})
    if which == "convdiff3d_64":
        seed = 3 if seed is None else seed
        nx = size or 64
        rng = np.random.default_rng(seed)
        csr = convdiff3d(nx)
        return _finish(which, csr, grid_coords((nx, nx, nx)), 128, 1e-3, 8, rng,
                       {"grid": (nx, nx, nx), "seed": seed})
    raise KeyError(which)


CONFIGS = ("poisson2d_32", "varcoef2d_256", "convdiff3d_64")


def make_batch(count=256, seed=4, leaf=64, eps=1e-4, nrhs=4):
    """Batch of independent systems (the batched-factorization workload).

    System i draws from its own child stream (seed, i): 2-D or 3-D with
    probability 1/2, grid side uniform in {64..256} (2-D) or {16..48} (3-D),
    diffusion with kappa = exp(N(0,1)) i.i.d. per cell (harmonic face means),
    leaf clusters of at most `leaf` points, epsilon 1e-4, nrhs uniform
    right-hand sides; about 9.0e6 unknowns in all for 256 systems.  Returns a
    list of Problem."""
    out = []
    for i in range(count):
        r = np.random.default_rng([seed, i])
        if r.random() < 0.5:
            s_ = int(r.integers(64, 257))
            csr = diffusion2d(np.exp(r.standard_normal(s_ * s_)), (s_, s_))
            co, grid = grid_coords((s_, s_)), (s_, s_)
        else:
            s_ = int(r.integers(16, 49))
            csr = diffusion3d(np.exp(r.standard_normal(s_ ** 3)), (s_, s_, s_))
            co, grid = grid_coords((s_, s_, s_)), (s_, s_, s_)
        out.append(_finish(f"batch{count}[{i}]", csr, co, leaf, eps, nrhs, r,
                           {"grid": grid, "seed": seed, "index": i}))
    return out


def make_serve_stream(count=2000, rate=200.0, seed=5, n_min=16384, n_max=262144):
    """Request stream of the serving workload (seeded).

    Poisson arrivals at `rate` per second.  20% factor requests (the first one
    always): type uniform over {2-D diffusion, 3-D diffusion, 2-D
    convection-diffusion w = (1, 0.5) 10, 3-D convection-diffusion
    w = (1, 0.5, 0.25) 10}, n uniform in [n_min, n_max] (grid side round(sqrt n)
    or round(cbrt n)), diffusion coefficients exp(N(0,1)) i.i.d., epsilon 1e-3 or
    1e-5, leaf 64 (2-D) or 128 (3-D).  80% solve requests: 1-32 right-hand sides
    uniform in [-1, 1] against a handle chosen uniformly among the factor
    requests issued so far.  Returns a list of dicts with keys t (arrival, s),
    kind ("factor" or "solve"), key, and for factors the matrix recipe
    (kind2, side, epsilon, leaf, seed) or for solves nrhs and rhs_seed; the
    matrices are built on demand by `build_serve_system`."""
    rng = np.random.default_rng(seed)
    t = np.cumsum(rng.exponential(1.0 / rate, count))
    reqs, factors = [], []
    types = ("diff2d", "diff3d", "convdiff2d", "convdiff3d")
    for i in range(count):
        if i == 0 or rng.random() < 0.2:
            typ = types[int(rng.integers(0, 4))]
            n = int(rng.integers(n_min, n_max + 1))
            side = int(round(n ** 0.5)) if typ.endswith("2d") else int(round(n ** (1.0 / 3.0)))
            eps = 1e-3 if rng.random() < 0.5 else 1e-5
            key = f"f{len(factors)}_{typ}_{side}_{eps:g}"
            factors.append(key)
            reqs.append({"t": float(t[i]), "kind": "factor", "key": key, "type": typ, "side": side,
                         "epsilon": eps, "leaf": 64 if typ.endswith("2d") else 128,
                         "seed": int(rng.integers(0, 2 ** 31))})
        else:
            reqs.append({"t": float(t[i]), "kind": "solve", "key": factors[int(rng.integers(0, len(factors)))],
                         "nrhs": int(rng.integers(1, 33)), "rhs_seed": int(rng.integers(0, 2 ** 31))})
    return reqs


def build_serve_system(req):
    """CSR matrix, cluster tree and epsilon of a factor request of
    make_serve_stream: returns (row_ptr, col_idx, val, perm, leaf_ptr, depth, eps)."""
    r = np.random.default_rng(req["seed"])
    s_ = req["side"]
    typ = req["type"]
    if typ == "diff2d":
        csr, co = diffusion2d(np.exp(r.standard_normal(s_ * s_)), (s_, s_)), grid_coords((s_, s_))
    elif typ == "diff3d":
        csr, co = diffusion3d(np.exp(r.standard_normal(s_ ** 3)), (s_, s_, s_)), grid_coords((s_, s_, s_))
    elif typ == "convdiff2d":
        csr, co = convdiff2d(s_), grid_coords((s_, s_))
    else:
        csr, co = convdiff3d(s_), grid_coords((s_, s_, s_))
    n = len(csr[0]) - 1
    depth = tree_depth(n, req["leaf"])
    perm, lp = rcb_tree(co, depth)
    return (*csr, perm, lp, depth, req["epsilon"])
