"""Helpers shared by the GPU parity tests (no test functions here).

Parity protocol for the FP64 mode (solutions, not stored blocks, are compared,
because V is unique only up to an orthogonal change of basis, Sec. 4.3):
  * the rank of every compression equals the oracle's; where one differs, every
    singular value between the two cuts lies at the threshold within the
    rounding band max(1e-8, 1e-13 / eps), and the oracle is re-run with the
    GPU's ranks (rank replay);
  * ||x_gpu - x_oracle|| / ||x_oracle|| <= 1e-10 for the stand-alone solve.
"""
import numpy as np

import oracle
from paper_1510_07363_amd import workloads as w

TOL = 1e-10


def grid(kind, nx, leaf, seed=0):
    rng = np.random.default_rng(seed)
    if kind == "poisson2d":
        csr, co = w.poisson2d(nx), w.grid_coords((nx, nx))
    elif kind == "varcoef2d":
        csr = w.diffusion2d(np.exp(w.gaussian_field_2d((nx, nx), rng, 8.0)), (nx, nx))
        co = w.grid_coords((nx, nx))
    elif kind == "convdiff3d":
        csr, co = w.convdiff3d(nx), w.grid_coords((nx, nx, nx))
    elif kind == "lognormal3d":
        csr = w.diffusion3d(np.exp(rng.standard_normal(nx ** 3)), (nx, nx, nx))
        co = w.grid_coords((nx, nx, nx))
    elif kind == "lognormal2d":
        csr = w.diffusion2d(np.exp(rng.standard_normal(nx * nx)), (nx, nx))
        co = w.grid_coords((nx, nx))
    elif kind == "convdiff2d":
        csr, co = w.convdiff2d(nx), w.grid_coords((nx, nx))
    else:
        raise KeyError(kind)
    n = len(csr[0]) - 1
    depth = w.tree_depth(n, leaf)
    perm, lp = w.rcb_tree(co, depth)
    return csr, n, perm, lp, depth, rng


def relerr(x, y):
    return np.linalg.norm(x - y) / np.linalg.norm(y)


def replay_ranks(gpu_ranks, Fo, eps, method="svd"):
    """None if every rank agrees, else the GPU's ranks as {(level, j): rank}
    after checking that each disagreement is a threshold tie: under eqn.
    cutOff1 every singular value between the two cuts lies at eps sigma_0, under
    the Frobenius rule (eqn. curOff6) every tail between them at eps N_i, within
    the rounding band max(1e-8, 1e-13 / eps)."""
    gpu = [int(r) for r in gpu_ranks]
    ora = [c.rank for c in Fo.compressions]
    assert len(gpu) == len(ora)
    if gpu == ora:
        return None
    assert method == "svd", "RRQR ranks must agree exactly on these inputs"
    band = max(1e-8, 1e-13 / eps)
    frob = getattr(Fo, "rule", "cutoff1") == "frob"
    top = max((float(c.sigma[0]) for c in Fo.compressions if len(c.sigma)), default=0.0)
    for rg, c in zip(gpu, Fo.compressions):
        if rg == c.rank:
            continue
        # a stacked block whose largest singular value is below 1e-8 of the largest
        # one is what remains of an exact cancellation (rounding noise): its rank is
        # not reproducible and carries no information; it is replayed
        if len(c.sigma) and method == "svd" and c.sigma[0] < 1e-8 * top:
            continue
        if frob:
            sig = np.asarray(c.sigma)
            tail = np.sqrt(np.concatenate([np.cumsum((sig ** 2)[::-1])[::-1], [0.0]]))
            tau = eps * Fo.level_norm[c.level]
            # the rank is the smallest k with tail_k < tau: the two sides disagree on
            # every k between their ranks, so each of those tails is at tau
            for k in range(min(rg, c.rank), max(rg, c.rank)):
                assert abs(tail[k] / tau - 1.0) <= band, (c.level, c.j, rg, c.rank, tail[k] / tau)
            continue
        sig = np.asarray(c.sigma) / c.sigma[0]
        for k in range(min(rg, c.rank), max(rg, c.rank)):
            assert abs(sig[k] / eps - 1.0) <= band, (c.level, c.j, rg, c.rank, sig[k])
    return {(c.level, c.j): rg for rg, c in zip(gpu, Fo.compressions)}


def oracle_matching(F, csr, perm, lp, depth, eps, Fo=None, order="colored", method="svd", rule="cutoff1",
                    **kw):
    """The oracle's factorization of the same input, rank-replayed onto the
    GPU handle F's ranks where they differ by a threshold tie.  A tie changes
    every later block, so the replay goes tie by tie: the first compression
    whose rank differs must be a tie (replay_ranks on it alone); the oracle is
    re-run with the GPU's ranks up to and including it, and compared again."""
    def run(forced):
        return oracle.factor(*csr, perm, lp, depth, eps, order=order, compress=method, check=False, rule=rule,
                             forced_ranks=forced, **kw)
    if Fo is None:
        Fo = run(None)
    if eps <= 1e-10:
        return Fo
    gpu = [int(r) for r in F.ranks()[0]]
    forced = {}
    for _ in range(64):
        diff = [q for q, c in enumerate(Fo.compressions) if gpu[q] != c.rank]
        if not diff:
            return Fo
        q = diff[0]
        # the first disagreement alone must be a threshold tie (or a noise block)
        only = [c.rank if k != q else gpu[q] for k, c in enumerate(Fo.compressions)]
        replay_ranks(only, Fo, eps, method)
        for k, c in enumerate(Fo.compressions[:q + 1]):
            forced[(c.level, c.j)] = gpu[k]
        Fo = run(dict(forced))
    raise AssertionError("rank replay did not converge")
