"""Serving loop (paper_1510_07363_amd.serve): scheduling, admission by HBM
budget, eviction and re-factor on demand, continuous batching of solves, and
"same result alone and in the mix".

The CPU tests run the scheduler over a backend built on the oracle (factor and
FGMRES in FP64 on the host, one right-hand side at a time), so batching cannot
change a result and alone/mix equality is exact.  The GPU test runs the same
scenarios on the library and bounds the alone/mix difference by the
conditioning (both answers reach the residual tolerance).
"""
import numpy as np
import pytest
import scipy.sparse as sp

import oracle
from paper_1510_07363_amd import workloads as w
from paper_1510_07363_amd.serve import OutOfBudget, Server, SystemSpec


def _spec(key, kind, nx, leaf, eps, seed):
    rng = np.random.default_rng(seed)
    if kind == "diff2d":
        csr = w.diffusion2d(np.exp(w.gaussian_field_2d((nx, nx), rng, 4.0)), (nx, nx))
        co = w.grid_coords((nx, nx))
    elif kind == "diff3d":
        csr = w.diffusion3d(np.exp(rng.standard_normal(nx ** 3)), (nx, nx, nx))
        co = w.grid_coords((nx, nx, nx))
    else:
        csr, co = w.convdiff2d(nx), w.grid_coords((nx, nx))
    n = len(csr[0]) - 1
    depth = w.tree_depth(n, leaf)
    perm, lp = w.rcb_tree(co, depth)
    return SystemSpec(key, *csr, perm, lp, depth, eps)


class OracleBackend:
    """Backend on the oracle: factor storage is charged at 800 bytes per unknown."""
    PER_UNKNOWN = 800
    WS_PER_UNKNOWN = 0            # workspace bytes per unknown and column charged by a round (tests set it)

    def __init__(self):
        self.factored, self.freed, self.batches, self.factor_batches = [], [], [], []
        self.trimmed, self.cycles = [], []

    def factor(self, spec, room):
        if spec.n * self.PER_UNKNOWN > room:
            raise OutOfBudget(f"{spec.key} needs {spec.n * self.PER_UNKNOWN} > {room}")
        F = oracle.factor(spec.row_ptr, spec.col_idx, spec.val, spec.perm, spec.leaf_ptr, spec.depth,
                          spec.epsilon, check=False)
        A = sp.csr_matrix((spec.val, spec.col_idx, spec.row_ptr), shape=(spec.n, spec.n))
        self.factored.append(spec.key)
        return {"key": spec.key, "F": F, "A": A, "n": spec.n}

    def factor_batch(self, specs, room):
        self.factor_batches.append([sp.key for sp in specs])
        return [self.factor(sp, room) for sp in specs]

    def resident_bytes(self, h):
        return h["n"] * self.PER_UNKNOWN + h.get("ws", 0)

    def trim(self, h):
        self.trimmed.append(h["key"])
        h["ws"] = 0

    def free(self, h):
        self.freed.append(h["key"])

    def solve_batch(self, items, nrhs, tol, restart, maxit, x0=False):
        """FGMRES per column; with x0, from the given iterate: the correction d
        solves A d = b - A x0 to the tolerance relative to ||b||."""
        self.batches.append(([h["key"] for h, _, _ in items], nrhs))
        self.cycles.append((restart, maxit, x0))
        out = []
        for h, B, X0 in items:
            h["ws"] = self.WS_PER_UNKNOWN * h["n"] * nrhs      # workspace grown by the round
            X = np.zeros_like(B)
            its = np.zeros(nrhs, dtype=np.int32)
            rr = np.zeros(nrhs)
            for k in range(nrhs):
                b = B[:, k]
                nb = np.linalg.norm(b)
                xs = X0[:, k] if x0 else np.zeros_like(b)
                if nb == 0.0:
                    X[:, k], its[k], rr[k] = 0.0, 0, 0.0
                    continue
                r0 = b - h["A"] @ xs
                nr0 = np.linalg.norm(r0)
                if nr0 <= tol * nb:
                    X[:, k], its[k], rr[k] = xs, 0, nr0 / nb
                    continue
                o = oracle.fgmres(h["A"], lambda v: oracle.solve(h["F"], v), r0, tol=tol * nb / nr0,
                                  restart=restart, maxit=maxit)
                X[:, k] = xs + o["x"]
                its[k] = o["iters"]
                rr[k] = np.linalg.norm(b - h["A"] @ X[:, k]) / nb
            out.append((X, its, rr))
        return out


SPECS = [("a", "diff2d", 16, 16, 1e-3, 1), ("b", "diff2d", 20, 16, 1e-3, 2), ("c", "convdiff", 16, 8, 1e-2, 3)]


def _server(budget_unknowns, **kw):
    be = OracleBackend()
    srv = Server(be, budget_unknowns * OracleBackend.PER_UNKNOWN, tol=1e-10, **kw)
    specs = {}
    for key, kind, nx, leaf, eps, seed in SPECS:
        s = _spec(key, kind, nx, leaf, eps, seed)
        srv.register(s)
        specs[key] = s
    return srv, be, specs


def test_continuous_batching_and_alone_equals_mix():
    rng = np.random.default_rng(0)
    srv, be, specs = _server(10_000)
    reqs = [("a", rng.uniform(-1, 1, specs["a"].n)), ("b", rng.uniform(-1, 1, (specs["b"].n, 3))),
            ("a", rng.uniform(-1, 1, (specs["a"].n, 2))), ("c", rng.uniform(-1, 1, specs["c"].n))]
    futs = [srv.submit(k, b) for k, b in reqs]
    srv.run_until_idle()
    # one round: factors admitted, then every request in one call per width class:
    # "c" (1 column) alone, "a" (its two requests, 1 + 2 columns) and "b" (3) padded to 4
    assert sorted(be.factored) == ["a", "b", "c"]
    assert srv.n_rounds == 1
    assert sorted((sorted(k), wd) for k, wd in be.batches) == [(["a", "b"], 4), (["c"], 1)]
    for (key, b), f in zip(reqs, futs):
        x, its, rr = f.result()
        assert x.shape == b.shape and (rr <= 1e-10).all()
        # the same request served alone gives the same answer
        srv2, _, _ = _server(10_000)
        f2 = srv2.submit(key, b)
        srv2.run_until_idle()
        x2, its2, rr2 = f2.result()
        assert np.array_equal(x, x2) and np.array_equal(its, its2)
        A = sp.csr_matrix((specs[key].val, specs[key].col_idx, specs[key].row_ptr), shape=(specs[key].n,) * 2)
        B = b.reshape(specs[key].n, -1)
        X = x.reshape(specs[key].n, -1)
        assert (np.linalg.norm(A @ X - B, axis=0) / np.linalg.norm(B, axis=0) <= 1e-10).all()
    st = srv.latency_stats()
    assert st["count"] == 4 and st["p99_ms"] >= st["p50_ms"] > 0


def test_admission_by_budget_evicts_idle_and_refactors_on_demand():
    rng = np.random.default_rng(1)
    # room for "b" (400 unknowns) or "a" + "c" (256 + 256), not all three
    srv, be, specs = _server(600)
    fa = srv.submit("a", rng.uniform(-1, 1, specs["a"].n))
    srv.run_until_idle()
    assert list(srv.resident) == ["a"]
    fb = srv.submit("b", rng.uniform(-1, 1, specs["b"].n))
    srv.run_until_idle()                                   # "a" is idle: evicted for "b"
    assert list(srv.resident) == ["b"] and be.freed == ["a"] and srv.n_evicted == 1
    assert srv.resident_bytes() <= srv.budget
    fa2 = srv.submit("a", rng.uniform(-1, 1, specs["a"].n))
    srv.run_until_idle()                                   # re-factored on demand
    assert be.factored == ["a", "b", "a"]
    for f in (fa, fb, fa2):
        assert (f.result()[2] <= 1e-10).all()


def test_admission_waits_for_busy_factor_then_serves():
    rng = np.random.default_rng(2)
    srv, be, specs = _server(600)
    srv.submit("b", rng.uniform(-1, 1, specs["b"].n))
    srv.step()                                             # "b" resident and served
    fb = srv.submit("b", rng.uniform(-1, 1, specs["b"].n))
    fa = srv.submit("a", rng.uniform(-1, 1, specs["a"].n))
    srv.step()       # "a" does not fit while "b" has a pending solve: "b" is served first
    assert fb.done() and not fa.done() and "a" not in srv.resident
    srv.run_until_idle()
    assert fa.done() and (fa.result()[2] <= 1e-10).all()


def test_request_too_large_fails_its_future_only():
    rng = np.random.default_rng(3)
    srv, be, specs = _server(300)                          # "b" (400 unknowns) never fits
    fb = srv.submit("b", rng.uniform(-1, 1, specs["b"].n))
    fa = srv.submit("a", rng.uniform(-1, 1, specs["a"].n))
    srv.run_until_idle()
    with pytest.raises(MemoryError):
        fb.result()
    assert (fa.result()[2] <= 1e-10).all()


def test_batch_limits_split_rounds():
    rng = np.random.default_rng(4)
    srv, be, specs = _server(10_000, max_batch_systems=2, max_width=4)
    futs = [srv.submit(k, rng.uniform(-1, 1, (specs[k].n, 3))) for k in ("a", "b", "c", "a")]
    srv.run_until_idle()
    assert all(len(keys) <= 2 for keys, _ in be.batches) and all(wd <= 4 for _, wd in be.batches)
    assert len(be.batches) >= 2
    for f in futs:
        assert (f.result()[2] <= 1e-10).all()


def test_factor_requests_and_worker_thread():
    """Factor requests complete with the factor's bytes; with the factor worker
    running (start), the same requests give the same answers as inline."""
    rng = np.random.default_rng(6)
    srv, be, specs = _server(10_000)
    srv.start()
    ff = [srv.submit_factor(k) for k in ("a", "b")]
    reqs = [(k, rng.uniform(-1, 1, (specs[k].n, 2))) for k in ("a", "b", "c", "a")]
    futs = [srv.submit(k, b) for k, b in reqs]
    srv.run_until_idle()
    srv.stop()
    assert [f.result() for f in ff] == [specs["a"].n * OracleBackend.PER_UNKNOWN,
                                       specs["b"].n * OracleBackend.PER_UNKNOWN]
    assert srv.latency_stats("factor")["count"] == 2
    srv2, _, _ = _server(10_000)
    f2 = [srv2.submit(k, b) for k, b in reqs]
    srv2.run_until_idle()
    for f, g in zip(futs, f2):
        assert np.array_equal(f.result()[0], g.result()[0])
    # a factor request for a resident system completes at once
    f3 = srv.submit_factor("a")
    assert f3.done() and f3.result() == specs["a"].n * OracleBackend.PER_UNKNOWN


def test_queued_factor_jobs_are_batched_by_epsilon():
    rng = np.random.default_rng(8)
    srv, be, specs = _server(10_000, max_factor_batch=4)
    # queue all jobs before the worker starts: "a" and "b" share epsilon 1e-3, "c" has 1e-2
    futs = [srv.submit(k, rng.uniform(-1, 1, specs[k].n)) for k in ("a", "c", "b")]
    srv.start()
    srv.run_until_idle()
    srv.stop()
    assert be.factor_batches == [["a", "b"]] and sorted(be.factored) == ["a", "b", "c"]
    for f in futs:
        assert (f.result()[2] <= 1e-10).all()


def test_failing_batched_factorization_falls_back_to_single_jobs():
    """A library error in a batched factorization (here raised by the backend)
    neither kills the factor worker nor leaves requests waiting: the jobs run one
    by one, and a job that fails alone fails only its own requests."""
    rng = np.random.default_rng(9)
    srv, be, specs = _server(10_000, max_factor_batch=4)

    def broken_batch(specs_, room):
        raise RuntimeError("device error in the batch")
    be.factor_batch = broken_batch
    single = be.factor

    def factor(spec, room):
        if spec.key == "b":
            raise RuntimeError("device error in b")
        return single(spec, room)
    be.factor = factor
    futs = {k: srv.submit(k, rng.uniform(-1, 1, specs[k].n)) for k in ("a", "b", "c")}
    srv.start()
    srv.run_until_idle()
    srv.stop()
    assert (futs["a"].result()[2] <= 1e-10).all() and (futs["c"].result()[2] <= 1e-10).all()
    with pytest.raises(RuntimeError):
        futs["b"].result()


def test_cancelled_requests_leave_the_queue():
    """A cancelled solve is dropped (its future reports cancelled, no round runs
    it), a cancelled factor request stops waiting, the other requests complete,
    and a completed request can no longer be cancelled."""
    rng = np.random.default_rng(10)
    srv, be, specs = _server(10_000)
    f_a = srv.submit("a", rng.uniform(-1, 1, specs["a"].n))
    f_b = srv.submit("b", rng.uniform(-1, 1, specs["b"].n))
    f_c = srv.submit("c", rng.uniform(-1, 1, specs["c"].n))
    f_fac = srv.submit_factor("c")
    assert srv.cancel(f_b) and f_b.cancelled()
    assert f_fac.cancel()                             # the plain Future API does the same
    srv.run_until_idle()
    assert (f_a.result()[2] <= 1e-10).all() and (f_c.result()[2] <= 1e-10).all()
    assert f_fac.cancelled()
    assert all("b" not in keys for keys, _ in be.batches)   # no round carried b's request
    assert not srv.cancel(f_a)


def test_submit_validation():
    srv, be, specs = _server(10_000)
    with pytest.raises(KeyError):
        srv.submit("zz", np.zeros(3))
    with pytest.raises(ValueError):
        srv.submit("a", np.zeros(specs["a"].n + 1))


@pytest.mark.gpu
def test_serve_on_gpu_alone_vs_mix():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    torch.cuda.set_device(0)
    from paper_1510_07363_amd.serve import LoraxBackend
    rng = np.random.default_rng(5)
    specs = [_spec("p", "diff2d", 48, 16, 1e-5, 11), _spec("q", "diff3d", 12, 32, 1e-3, 12),
             _spec("r", "convdiff", 40, 16, 1e-3, 13)]
    srv = Server(LoraxBackend(precision="mixed"), 8 << 30, tol=1e-10)
    for s in specs:
        srv.register(s)
    reqs = [(s.key, rng.uniform(-1, 1, (s.n, k))) for s, k in zip(specs, (1, 5, 2))]
    reqs.append(("p", rng.uniform(-1, 1, (specs[0].n, 3))))
    futs = [srv.submit(k, b) for k, b in reqs]
    srv.run_until_idle()
    assert srv.batches == [3] and srv.n_factored == 3
    bykey = {s.key: s for s in specs}
    for (key, b), f in zip(reqs, futs):
        x, its, rr = f.result()
        s = bykey[key]
        A = sp.csr_matrix((s.val, s.col_idx, s.row_ptr), shape=(s.n, s.n))
        r_mix = np.linalg.norm(A @ x - b, axis=0) / np.linalg.norm(b, axis=0)
        assert (r_mix <= 1e-10).all() and (rr <= 1e-10).all()
        # alone: the same request through the same server (factor resident)
        f1 = srv.submit(key, b)
        srv.run_until_idle()
        x1 = f1.result()[0]
        r1 = np.linalg.norm(A @ x1 - b, axis=0) / np.linalg.norm(b, axis=0)
        smin = np.linalg.svd(A.toarray(), compute_uv=False)[-1]
        bound = (r_mix + r1) * np.linalg.norm(b, axis=0) / smin
        assert (np.linalg.norm(x - x1, axis=0) <= 1.01 * bound + 1e-14).all()
    st = srv.latency_stats()
    assert st["count"] == 8
    srv.close()
    assert srv.resident_bytes() == 0


@pytest.mark.gpu
def test_serve_on_gpu_concurrent_factoring():
    """Factor jobs on a worker thread and stream of their own while solve rounds
    run on another stream; every answer reaches the tolerance."""
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    torch.cuda.set_device(0)
    from paper_1510_07363_amd.serve import LoraxBackend
    rng = np.random.default_rng(7)
    specs = [_spec("p", "diff2d", 64, 16, 1e-3, 21), _spec("q", "diff3d", 14, 32, 1e-3, 22),
             _spec("r", "convdiff", 48, 16, 1e-3, 23), _spec("s", "diff2d", 40, 16, 1e-5, 24)]
    srv = Server(LoraxBackend(precision="mixed"), 8 << 30, tol=1e-10,
                 factor_backend=LoraxBackend(precision="mixed"))
    for s_ in specs:
        srv.register(s_)
    srv.start()
    ff = [srv.submit_factor(s_.key) for s_ in specs]
    reqs = [(s_.key, rng.uniform(-1, 1, (s_.n, k))) for s_, k in zip(specs * 2, (1, 4, 2, 3, 5, 1, 2, 8))]
    futs = [srv.submit(k, b) for k, b in reqs]
    srv.run_until_idle()
    srv.stop()
    assert all(f.result() > 0 for f in ff)
    bykey = {s_.key: s_ for s_ in specs}
    for (key, b), f in zip(reqs, futs):
        x, its, rr = f.result()
        s_ = bykey[key]
        A = sp.csr_matrix((s_.val, s_.col_idx, s_.row_ptr), shape=(s_.n, s_.n))
        assert (np.linalg.norm(A @ x - b, axis=0) / np.linalg.norm(b, axis=0) <= 1e-10).all()
    assert srv.latency_stats("solve")["count"] == len(reqs)
    srv.close()



def test_cycle_rounds_admit_new_requests_between_cycles():
    """With cycle = 2, a round is one FGMRES(2) cycle: unconverged right-hand
    sides carry their iterate into the next round (initial guess), and a
    request submitted after the first round joins the second, beside them.
    Every answer reaches the tolerance and equals the same request served
    alone (the fake backend works column by column, so the mix cannot change
    the arithmetic)."""
    rng = np.random.default_rng(11)
    srv, be, specs = _server(10_000, cycle=2)
    b1 = rng.uniform(-1, 1, (specs["c"].n, 2))
    b2 = rng.uniform(-1, 1, specs["b"].n)
    f1 = srv.submit("c", b1)
    srv.step()                                  # factor "c", first cycle of f1
    assert not f1.done() and srv.n_rounds == 1
    f2 = srv.submit("b", b2)                    # arrives between cycles
    srv.run_until_idle()
    assert all(c == (2, 2, True) for c in be.cycles)
    second = be.batches[1:]
    assert any("b" in keys for keys, _ in second) and any("c" in keys for keys, _ in second)
    for key, b, f in (("c", b1, f1), ("b", b2, f2)):
        x, its, rr = f.result()
        A = sp.csr_matrix((specs[key].val, specs[key].col_idx, specs[key].row_ptr), shape=(specs[key].n,) * 2)
        X, B = x.reshape(specs[key].n, -1), b.reshape(specs[key].n, -1)
        assert (np.linalg.norm(A @ X - B, axis=0) / np.linalg.norm(B, axis=0) <= 1e-10).all() and (rr <= 1e-10).all()
        assert (its > 2).any()                  # more than one cycle was needed
        srv2, _, _ = _server(10_000, cycle=2)
        g = srv2.submit(key, b)
        srv2.run_until_idle()
        assert np.array_equal(g.result()[0], x) and np.array_equal(g.result()[1], its)


def test_round_workspace_counts_in_admission():
    """A round reserves its GMRES workspace: idle handles are trimmed first,
    then idle systems evicted when the footprint would exceed the budget."""
    rng = np.random.default_rng(12)
    OracleBackend.WS_PER_UNKNOWN = 100
    try:
        srv, be, specs = _server(900)          # 720,000 bytes
        fa = srv.submit("a", rng.uniform(-1, 1, (specs["a"].n, 1)))
        srv.run_until_idle()                   # "a": 256 unknowns -> 204,800 bytes + 25,600 of workspace
        assert srv.resident["a"].bytes == 256 * 800 + 256 * 100
        fc = srv.submit("c", rng.uniform(-1, 1, (specs["c"].n, 4)))
        srv.run_until_idle()                   # "c" factored; its 4-column round needs room
        assert "a" in be.trimmed               # the idle handle gave its workspace back first
        assert srv.resident_bytes() <= srv.budget
        fb = srv.submit("b", rng.uniform(-1, 1, (specs["b"].n, 8)))
        srv.run_until_idle()                   # 400 unknowns + an 8-column workspace: idle systems go
        assert srv.n_evicted >= 1 and srv.resident_bytes() <= srv.budget
        for f in (fa, fc, fb):
            assert (f.result()[2] <= 1e-10).all()
    finally:
        OracleBackend.WS_PER_UNKNOWN = 0
