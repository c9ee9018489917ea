"""Serving loop over resident factorizations (factor once, solve many times).

A Server keeps factorizations resident in HBM under a byte budget and answers
solve requests with FGMRES preconditioned by the factorization (the use the
paper makes of one factorization for many right-hand sides, Sec. 6.2).  Work is
scheduled in rounds (`step`):

* admission: a solve request whose system is not resident queues a factor job;
  a factor job runs when the resident factors plus its own storage fit the
  budget.  The budget is enforced by the library itself (the factor's
  hbm_budget_bytes is the room left, so an oversized factor fails with
  LRX_ENOMEM instead of overcommitting); on that failure idle resident factors
  are evicted, least recently used first, and the job is retried, or it waits
  while solves on resident factors are still pending, or its requests fail
  when nothing more can be freed.
* continuous batching: all ready solve requests, over every resident system,
  go into one lrx_gmres_batch_dev call per round (several requests on one
  system are concatenated as extra right-hand sides; every system's block is
  padded with zero columns to the batch's width, rounded up to a power of two).
  A request's result does not depend on which other systems share its batch;
  the width of the batch changes only the summation order of its dot products.
* completion: each request's future receives (x, iterations, relative
  residuals); its latency (completion - arrival) is recorded.

The arithmetic runs in the library (the backend); this module only schedules,
marshals arrays and measures.  PyTorch provides device memory and the stream.
"""
from __future__ import annotations

import collections
import concurrent.futures as cf
import time
from dataclasses import dataclass, field

import numpy as np

__all__ = ["SystemSpec", "SolveRequest", "Server", "LoraxBackend"]


@dataclass
class SystemSpec:
    """A linear system the server may be asked to solve: CSR matrix and cluster tree."""
    key: str
    row_ptr: np.ndarray
    col_idx: np.ndarray
    val: np.ndarray
    perm: np.ndarray
    leaf_ptr: np.ndarray
    depth: int
    epsilon: float

    @property
    def n(self) -> int:
        return len(self.row_ptr) - 1


@dataclass
class SolveRequest:
    key: str
    b: np.ndarray                       # (n,) or (n, k)
    arrival: float = field(default_factory=time.perf_counter)
    future: cf.Future = field(default_factory=cf.Future)


class OutOfBudget(Exception):
    """The factorization does not fit in the room left under the budget."""


class LoraxBackend:
    """The library on the current GPU: lrx_factor for factor jobs and
    lrx_gmres_batch_dev for each batch of solves, on one stream."""

    def __init__(self, precision="mixed", stream=None):
        import torch
        from . import lorax
        self.torch, self.lx = torch, lorax
        self.precision = precision
        self.stream = stream
        self.device = "cuda:%d" % torch.cuda.current_device()

    def factor(self, spec: SystemSpec, room_bytes: int):
        lx = self.lx
        sptr = self.stream.cuda_stream if self.stream is not None else None
        try:
            return lx.Factor(spec.row_ptr, spec.col_idx, spec.val, spec.perm, spec.leaf_ptr, spec.depth,
                             spec.epsilon, stream=sptr, hbm_budget_bytes=max(int(room_bytes), 1),
                             precision=self.precision)
        except lx.LoraxError as e:
            if e.status == lx.LRX_ENOMEM:
                raise OutOfBudget(str(e)) from None
            raise

    def resident_bytes(self, handle) -> int:
        return int(handle.stats()["factor_bytes"])

    def free(self, handle) -> None:
        handle.free()

    def solve_batch(self, items, nrhs, tol, restart, maxit):
        """items: list of (handle, B) with B of shape (n, nrhs); returns a list of
        (X, iters, relres) in the same order."""
        torch, lx = self.torch, self.lx
        bs = [torch.from_numpy(np.ascontiguousarray(B.T)).to(self.device) for _, B in items]
        xs = [torch.zeros_like(b) for b in bs]
        its, rr, st = lx.gmres_batch_dev([h for h, _ in items], nrhs, [b.data_ptr() for b in bs],
                                         [x.data_ptr() for x in xs], tol=tol, restart=restart, maxit=maxit)
        return [(x.cpu().numpy().T, its[i], rr[i]) for i, x in enumerate(xs)]


class _Resident:
    __slots__ = ("handle", "bytes", "last_use")

    def __init__(self, handle, nbytes, t):
        self.handle, self.bytes, self.last_use = handle, nbytes, t


class Server:
    def __init__(self, backend, hbm_budget_bytes, tol=1e-10, restart=30, maxit=500, max_batch_systems=256,
                 max_width=256):
        if hbm_budget_bytes <= 0:
            raise ValueError("hbm_budget_bytes must be positive")
        self.backend = backend
        self.budget = int(hbm_budget_bytes)
        self.tol, self.restart, self.maxit = tol, restart, maxit
        self.max_batch_systems = max_batch_systems
        self.max_width = max_width
        self.specs: dict[str, SystemSpec] = {}
        self.resident: "collections.OrderedDict[str, _Resident]" = collections.OrderedDict()
        self.pending: "collections.deque[SolveRequest]" = collections.deque()
        self.latencies: list[float] = []
        self.n_solved = 0
        self.n_factored = 0
        self.n_evicted = 0
        self.batches: list[int] = []              # systems per solve batch

    # ------------------------------------------------------------ interface
    def register(self, spec: SystemSpec) -> None:
        self.specs[spec.key] = spec

    def submit(self, key: str, b, arrival: float | None = None) -> cf.Future:
        if key not in self.specs:
            raise KeyError(f"unknown system {key!r}")
        b = np.asarray(b, dtype=np.float64)
        n = self.specs[key].n
        if b.shape[0] != n or b.ndim not in (1, 2):
            raise ValueError(f"b must have {n} rows")
        req = SolveRequest(key, b) if arrival is None else SolveRequest(key, b, arrival)
        self.pending.append(req)
        return req.future

    def evict(self, key: str) -> bool:
        """Frees the factorization of key (it is factored again on demand)."""
        r = self.resident.pop(key, None)
        if r is None:
            return False
        self.backend.free(r.handle)
        self.n_evicted += 1
        return True

    def resident_bytes(self) -> int:
        return sum(r.bytes for r in self.resident.values())

    def step(self) -> int:
        """One scheduling round; returns the number of requests completed."""
        if not self.pending:
            return 0
        self._admit()
        return self._solve_ready()

    def run_until_idle(self, max_rounds=1_000_000) -> None:
        for _ in range(max_rounds):
            if not self.pending:
                return
            self.step()
        raise RuntimeError("server did not drain")

    def latency_stats(self) -> dict:
        if not self.latencies:
            return {"count": 0}
        lat = np.array(self.latencies)
        return {"count": int(lat.size), "p50_ms": float(np.percentile(lat, 50) * 1e3),
                "p99_ms": float(np.percentile(lat, 99) * 1e3), "mean_ms": float(lat.mean() * 1e3)}

    def close(self) -> None:
        for key in list(self.resident):
            self.evict(key)

    # ------------------------------------------------------------ internals
    def _admit(self) -> None:
        needed = []
        for req in self.pending:
            if req.key not in self.resident and req.key not in needed:
                needed.append(req.key)
        busy = {req.key for req in self.pending if req.key in self.resident}
        for key in needed:
            spec = self.specs[key]
            while True:
                room = self.budget - self.resident_bytes()
                try:
                    h = self.backend.factor(spec, room) if room > 0 else None
                    if h is None:
                        raise OutOfBudget("no room left")
                except OutOfBudget:
                    idle = [k for k in self.resident if k not in busy]
                    if idle:
                        self.evict(idle[0])                 # least recently used first
                        continue
                    if busy:
                        break                               # wait for solves in flight to finish
                    self._fail_key(key, MemoryError(f"system {key} does not fit in the HBM budget"))
                    break
                except Exception as e:                      # a library error: fail its requests
                    self._fail_key(key, e)
                    break
                self.resident[key] = _Resident(h, self.backend.resident_bytes(h), time.perf_counter())
                self.n_factored += 1
                break

    def _fail_key(self, key, exc) -> None:
        keep = collections.deque()
        for req in self.pending:
            if req.key == key:
                req.future.set_exception(exc)
            else:
                keep.append(req)
        self.pending = keep

    def _solve_ready(self) -> int:
        # requests of resident systems, grouped by system, up to the batch limits
        groups: "collections.OrderedDict[str, list[SolveRequest]]" = collections.OrderedDict()
        width: dict[str, int] = {}
        rest = collections.deque()
        for req in self.pending:
            k = 1 if req.b.ndim == 1 else req.b.shape[1]
            if req.key not in self.resident:
                rest.append(req)
                continue
            if req.key not in groups and len(groups) >= self.max_batch_systems:
                rest.append(req)
                continue
            if width.get(req.key, 0) + k > self.max_width:
                rest.append(req)
                continue
            groups.setdefault(req.key, []).append(req)
            width[req.key] = width.get(req.key, 0) + k
        self.pending = rest
        if not groups:
            return 0
        w = max(width.values())
        nrhs = 1
        while nrhs < w:
            nrhs *= 2
        items, spans = [], []
        for key, reqs in groups.items():
            n = self.specs[key].n
            B = np.zeros((n, nrhs))
            c0, sp = 0, []
            for req in reqs:
                k = 1 if req.b.ndim == 1 else req.b.shape[1]
                B[:, c0:c0 + k] = req.b.reshape(n, k)
                sp.append((req, c0, k))
                c0 += k
            items.append((self.resident[key].handle, B))
            spans.append(sp)
        try:
            out = self.backend.solve_batch(items, nrhs, self.tol, self.restart, self.maxit)
        except Exception as e:
            for sp in spans:
                for req, _, _ in sp:
                    req.future.set_exception(e)
            return 0
        now = time.perf_counter()
        done = 0
        for key, sp, (X, its, rr) in zip(groups, spans, out):
            self.resident[key].last_use = now
            self.resident.move_to_end(key)
            for req, c0, k in sp:
                x = X[:, c0:c0 + k]
                res = (x[:, 0] if req.b.ndim == 1 else x.copy(), np.asarray(its[c0:c0 + k]),
                       np.asarray(rr[c0:c0 + k]))
                self.latencies.append(now - req.arrival)
                req.future.set_result(res)
                done += 1
        self.n_solved += done
        self.batches.append(len(groups))
        return done
