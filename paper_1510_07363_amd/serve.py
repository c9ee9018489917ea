"""Serving loop over resident factorizations (factor once, solve many times).

A Server keeps factorizations resident in HBM under a byte budget and answers
factor and solve requests; solves use FGMRES preconditioned by the
factorization (the use the paper makes of one factorization for many
right-hand sides, Sec. 6.2).

* admission: a factor request, or a solve request whose system is not
  resident, queues a factor job.  A factor job runs when the resident factors
  plus its own storage fit the budget.  The budget is enforced by the library
  itself (the factor's hbm_budget_bytes is the room left, so an oversized
  factor fails with LRX_ENOMEM instead of overcommitting); on that failure idle
  resident factors are evicted, least recently used first, and the job is
  retried, or it waits while solves on resident factors are in flight, or its
  requests fail when nothing more can be freed.
* admission counts device footprints: a resident system is charged what its
  handle holds on the device (factor storage, solve programs, resident A and
  the solve / GMRES workspaces it has grown to: lrx_stats device_bytes), and a
  solve round first reserves the Krylov workspace it will grow, trimming the
  workspaces of idle handles and then evicting idle systems when the budget
  would be exceeded.  A round that still runs out of device memory evicts the
  idle systems and is retried once.
* continuous batching: each round puts the ready solve requests, over every
  resident system, into batched FGMRES calls (several requests on one system
  are concatenated as extra right-hand sides).  Systems are grouped by width
  class (their own column count rounded up to a power of two), one call per
  class, so a one-column request is never padded to the widest system's
  width.  With `cycle` set, a round is one FGMRES restart cycle of `cycle`
  Arnoldi steps: right-hand sides that have not converged carry their iterate
  into the next round as its initial guess (lrx_gmres_batch_dev_x0), next to
  requests that arrived meanwhile, so new work is admitted every `cycle` steps
  instead of after whole solves.  Without `cycle` a round solves to
  convergence (FGMRES(restart)).  A request's result does not depend on which
  other systems share its batch; the width of its class changes only the
  summation order of its dot products.
* overlap: with `start()`, factor jobs run on a worker thread with their own
  backend (its own stream), so factorizations and solve rounds proceed on the
  device at the same time; without it, `step()` runs factor jobs inline.
* completion: each request's future receives its result, (x, iterations,
  relative residuals) for solves and the factor's byte count for factors; its
  latency (completion - arrival) is recorded by kind.

The arithmetic runs in the library (the backend); this module only schedules,
marshals arrays and measures.  PyTorch provides device memory and streams.
"""
from __future__ import annotations

import collections
import concurrent.futures as cf
import threading
import time
from dataclasses import dataclass, field

import numpy as np

__all__ = ["SystemSpec", "Server", "LoraxBackend", "OutOfBudget"]


@dataclass
class SystemSpec:
    """A linear system the server may be asked to factor and solve: CSR matrix and cluster tree."""
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
class _Request:
    kind: str                           # "solve" or "factor"
    key: str
    b: np.ndarray | None
    arrival: float
    future: cf.Future = field(default_factory=cf.Future)
    # solves, across rounds: iterate, iterations, relative residuals, converged flags (per column)
    x: np.ndarray | None = None
    its: np.ndarray | None = None
    rr: np.ndarray | None = None
    conv: np.ndarray | None = None

    def cols(self) -> int:
        return 1 if self.b.ndim == 1 else self.b.shape[1]


class OutOfBudget(Exception):
    """The factorization does not fit in the room left under the budget."""


class LoraxBackend:
    """The library on the current GPU: lrx_factor for factor jobs and
    lrx_gmres_batch_dev for each batch of solves, on one stream (None: a new
    stream of default priority)."""

    def __init__(self, precision="mixed", stream=None):
        import torch
        from . import lorax
        self.torch, self.lx = torch, lorax
        self.precision = precision
        self.device_index = torch.cuda.current_device()
        self.device = "cuda:%d" % self.device_index
        self.stream = stream if stream is not None else torch.cuda.Stream(device=self.device)

    def factor(self, spec: SystemSpec, room_bytes: int):
        lx, torch = self.lx, self.torch
        torch.cuda.set_device(self.device_index)          # worker threads start on device 0
        try:
            return lx.Factor(spec.row_ptr, spec.col_idx, spec.val, spec.perm, spec.leaf_ptr, spec.depth,
                             spec.epsilon, stream=self.stream.cuda_stream,
                             hbm_budget_bytes=max(int(room_bytes), 1), precision=self.precision)
        except lx.LoraxError as e:
            if e.status == lx.LRX_ENOMEM:
                raise OutOfBudget(str(e)) from None
            raise

    def factor_batch(self, specs, room_bytes: int):
        """Several systems of one epsilon in one lrx_factor_batch call; each
        handle's storage is capped at room_bytes (LRX_ENOMEM: OutOfBudget)."""
        lx, torch = self.lx, self.torch
        torch.cuda.set_device(self.device_index)
        try:
            return lx.factor_batch([(sp.row_ptr, sp.col_idx, sp.val, sp.perm, sp.leaf_ptr, sp.depth)
                                    for sp in specs], specs[0].epsilon, stream=self.stream.cuda_stream,
                                   hbm_budget_bytes=max(int(room_bytes), 1), precision=self.precision)
        except lx.LoraxError as e:
            if e.status == lx.LRX_ENOMEM:
                raise OutOfBudget(str(e)) from None
            raise

    def resident_bytes(self, handle) -> int:
        """Device bytes the handle holds now (factor, programs, A, workspaces)."""
        return int(handle.stats()["device_bytes"])

    def trim(self, handle) -> None:
        """Releases the handle's solve/GMRES workspaces (the factor stays)."""
        handle.trim()

    def adopt(self, handle) -> None:
        """A handle factored elsewhere is solved on this backend's stream."""
        handle.set_stream(self.stream.cuda_stream)

    def free(self, handle) -> None:
        handle.free()

    def solve_batch(self, items, nrhs, tol, restart, maxit, x0=False):
        """items: list of (handle, B, X0) with B of shape (n, nrhs) and X0 the
        initial guess (same shape) when x0 is set (else ignored); returns a list
        of (X, iters, relres) in the same order.  Out of device memory raises
        OutOfBudget."""
        torch, lx = self.torch, self.lx
        torch.cuda.set_device(self.device_index)
        with torch.cuda.stream(self.stream):
            bs = [torch.from_numpy(np.ascontiguousarray(B.T)).to(self.device) for _, B, _ in items]
            if x0:
                xs = [torch.from_numpy(np.ascontiguousarray(X0.T)).to(self.device) for _, _, X0 in items]
            else:
                xs = [torch.zeros_like(b) for b in bs]
            self.stream.synchronize()
            # the library runs the batch on the stream of the first handle; the
            # inputs above are complete before it starts
            try:
                its, rr, st = lx.gmres_batch_dev([h for h, _, _ in items], nrhs, [b.data_ptr() for b in bs],
                                                 [x.data_ptr() for x in xs], tol=tol, restart=restart,
                                                 maxit=maxit, x0=x0)
            except lx.LoraxError as e:
                if e.status == lx.LRX_ENOMEM:
                    raise OutOfBudget(str(e)) from None
                raise
            out = [(x.cpu().numpy().T, its[i], rr[i]) for i, x in enumerate(xs)]
        return out


class _Resident:
    __slots__ = ("handle", "bytes", "last_use")

    def __init__(self, handle, nbytes, t):
        self.handle, self.bytes, self.last_use = handle, nbytes, t


class Server:
    def __init__(self, backend, hbm_budget_bytes, tol=1e-10, restart=30, maxit=500, max_batch_systems=256,
                 max_width=256, factor_backend=None, max_factor_batch=1, cycle=None):
        if hbm_budget_bytes <= 0:
            raise ValueError("hbm_budget_bytes must be positive")
        self.backend = backend
        self.factor_backend = factor_backend if factor_backend is not None else backend
        self.budget = int(hbm_budget_bytes)
        self.tol, self.restart, self.maxit = tol, restart, maxit
        self.max_batch_systems = max_batch_systems
        self.max_width = max_width
        self.max_factor_batch = max_factor_batch
        if cycle is not None and not (1 <= int(cycle) <= restart):
            raise ValueError("cycle must be in [1, restart]")
        self.cycle = None if cycle is None else int(cycle)
        self.n_rounds = 0
        self.specs: dict[str, SystemSpec] = {}
        self.resident: "collections.OrderedDict[str, _Resident]" = collections.OrderedDict()
        self.pending: "collections.deque[_Request]" = collections.deque()     # solves
        self.factor_waiters: dict[str, list] = {}                            # factor requests by key
        self.jobs: "collections.deque[str]" = collections.deque()            # factor jobs to run
        self.factoring: set[str] = set()                                     # factor jobs running
        self.busy: set[str] = set()                                          # systems in a solve round
        self.latencies: dict[str, list] = {"solve": [], "factor": []}
        self.n_solved = 0
        self.n_factored = 0
        self.n_evicted = 0
        self.batches: list[int] = []              # systems per solve round
        self._lock = threading.Lock()
        self._wake = threading.Condition(self._lock)
        self._worker = None
        self._stop = False

    # ------------------------------------------------------------ interface
    def register(self, spec: SystemSpec) -> None:
        with self._lock:
            self.specs[spec.key] = spec

    def submit(self, key: str, b, arrival: float | None = None) -> cf.Future:
        """Solve request: future of (x, iterations, relative residuals)."""
        b = np.asarray(b, dtype=np.float64)
        with self._lock:
            if key not in self.specs:
                raise KeyError(f"unknown system {key!r}")
            n = self.specs[key].n
            if b.shape[0] != n or b.ndim not in (1, 2):
                raise ValueError(f"b must have {n} rows")
            req = _Request("solve", key, b, time.perf_counter() if arrival is None else arrival)
            self.pending.append(req)
            self._need(key)
            self._wake.notify_all()
        return req.future

    def submit_factor(self, key: str, arrival: float | None = None) -> cf.Future:
        """Factor request: future of the resident factor's byte count."""
        with self._lock:
            if key not in self.specs:
                raise KeyError(f"unknown system {key!r}")
            req = _Request("factor", key, None, time.perf_counter() if arrival is None else arrival)
            if key in self.resident:
                self._complete_factor(req, self.resident[key].bytes)
            else:
                self.factor_waiters.setdefault(key, []).append(req)
                self._need(key)
                self._wake.notify_all()
        return req.future

    def evict(self, key: str) -> bool:
        """Frees the factorization of key (it is factored again on demand)."""
        with self._lock:
            return self._evict(key)

    def resident_bytes(self) -> int:
        with self._lock:
            return self._resident_bytes()

    def start(self) -> None:
        """Runs factor jobs on a worker thread (overlapping the solve rounds)."""
        if self._worker is None:
            self._stop = False
            self._worker = threading.Thread(target=self._factor_loop, daemon=True)
            self._worker.start()

    def stop(self) -> None:
        if self._worker is not None:
            with self._lock:
                self._stop = True
                self._wake.notify_all()
            self._worker.join()
            self._worker = None

    def step(self) -> int:
        """One scheduling round: factor jobs (inline unless the worker runs), then
        one batch of ready solves.  Returns the number of requests completed."""
        done = 0
        if self._worker is None:
            with self._lock:
                njobs = len(self.jobs)
            for _ in range(njobs):                      # a job that must wait goes back to the queue
                with self._lock:
                    if not self.jobs:
                        break
                    key = self.jobs.popleft()
                    self.factoring.add(key)
                done += self._run_factor_job(key, inline=True)
        return done + self._solve_ready()

    def idle(self) -> bool:
        with self._lock:
            return not self.pending and not self.jobs and not self.factoring and not self.factor_waiters

    def run_until_idle(self, max_rounds=10_000_000) -> None:
        for _ in range(max_rounds):
            if self.idle():
                return
            if self.step() == 0 and self._worker is not None:
                with self._lock:
                    if not self._ready_keys():
                        self._wake.wait(timeout=0.005)
        raise RuntimeError("server did not drain")

    def latency_stats(self, kind="solve") -> dict:
        with self._lock:
            lat = np.array(self.latencies[kind])
        if lat.size == 0:
            return {"count": 0}
        return {"count": int(lat.size), "p50_ms": float(np.percentile(lat, 50) * 1e3),
                "p99_ms": float(np.percentile(lat, 99) * 1e3), "mean_ms": float(lat.mean() * 1e3)}

    def close(self) -> None:
        self.stop()
        with self._lock:
            for key in list(self.resident):
                self._evict(key)

    # ------------------------------------------------------------ internals (lock held)
    def _resident_bytes(self) -> int:
        return sum(r.bytes for r in self.resident.values())

    def _need(self, key) -> None:
        if key not in self.resident and key not in self.factoring and key not in self.jobs:
            self.jobs.append(key)

    def _evict(self, key) -> bool:
        r = self.resident.pop(key, None)
        if r is None:
            return False
        self.backend.free(r.handle)
        self.n_evicted += 1
        return True

    def cancel(self, future: cf.Future) -> bool:
        """Cancels a request that has not completed (Future.cancel has the same
        effect): a queued solve leaves the queue at the next round, one in a
        running round is dropped when the round ends (its partial iterate is
        discarded), a factor request stops waiting (the factorization itself
        goes on for the other requests of that system).  False if the request
        has already completed."""
        ok = future.cancel()
        if ok:
            with self._lock:
                self._wake.notify_all()
        return ok

    def _complete_factor(self, req, nbytes) -> None:
        if req.future.cancelled():
            return
        self.latencies["factor"].append(time.perf_counter() - req.arrival)
        req.future.set_result(nbytes)

    def _fail_key(self, key, exc) -> None:
        keep = collections.deque()
        for req in self.pending:
            if req.key == key:
                if not req.future.cancelled():
                    req.future.set_exception(exc)
            else:
                keep.append(req)
        self.pending = keep
        for req in self.factor_waiters.pop(key, []):
            if not req.future.cancelled():
                req.future.set_exception(exc)

    def _ready_keys(self):
        return [r.key for r in self.pending if r.key in self.resident and r.key not in self.busy]

    # ------------------------------------------------------------ factor jobs
    def _factor_loop(self) -> None:
        while True:
            with self._lock:
                while not self.jobs and not self._stop:
                    self._wake.wait()
                if self._stop:
                    return
                key = self.jobs.popleft()
                # queued jobs of the same epsilon join one batched factorization
                group = [key]
                if self.max_factor_batch > 1 and hasattr(self.factor_backend, "factor_batch"):
                    eps = self.specs[key].epsilon
                    for k in list(self.jobs):
                        if len(group) >= self.max_factor_batch:
                            break
                        if self.specs[k].epsilon == eps:
                            self.jobs.remove(k)
                            group.append(k)
                self.factoring |= set(group)
            try:
                if len(group) == 1 or not self._run_factor_batch(group):
                    for k in group:
                        self._run_factor_job(k, inline=False)
            except Exception as e:                          # the worker must not die silently
                with self._lock:
                    for k in group:
                        if k not in self.resident:
                            self._fail_key(k, e)
                    self.factoring -= set(group)
                    self._wake.notify_all()

    def _run_factor_batch(self, group) -> bool:
        """One lrx_factor_batch over group; False (nothing admitted) when it does
        not fit, the jobs then run one by one."""
        with self._lock:
            room = self.budget - self._resident_bytes()
            specs = [self.specs[k] for k in group]
        if room <= 0:
            return False
        try:
            hs = self.factor_backend.factor_batch(specs, room)
        except OutOfBudget:
            return False
        except Exception:                                   # a library error: one by one, each job
            return False                                    # fails (or succeeds) on its own
        for h in hs:
            if self.factor_backend is not self.backend and hasattr(self.backend, "adopt"):
                self.backend.adopt(h)
        with self._lock:
            for k, h in zip(group, hs):
                nbytes = self.factor_backend.resident_bytes(h)
                self.resident[k] = _Resident(h, nbytes, time.perf_counter())
                self.n_factored += 1
                for req in self.factor_waiters.pop(k, []):
                    self._complete_factor(req, nbytes)
            # each handle was capped at the room left; the batch as a whole may
            # exceed it: idle systems outside the batch are evicted to compensate
            wanted = {r.key for r in self.pending} | self.busy | set(group)
            while self._resident_bytes() > self.budget:
                idle = [k for k in self.resident if k not in wanted]
                if not idle:
                    break
                self._evict(idle[0])
            self.factoring -= set(group)
            self._wake.notify_all()
        return True

    def _run_factor_job(self, key, inline) -> int:
        """Factors key under the budget (evicting idle systems as needed).
        Returns the number of factor requests completed."""
        spec = self.specs[key]
        while True:
            with self._lock:
                room = self.budget - self._resident_bytes()
            try:
                if room <= 0:
                    raise OutOfBudget("no room left")
                h = self.factor_backend.factor(spec, room)
            except OutOfBudget:
                with self._lock:
                    # systems with pending or running solves are kept
                    wanted = {r.key for r in self.pending} | self.busy
                    idle = [k for k in self.resident if k not in wanted]
                    if idle:
                        self._evict(idle[0])                # least recently used first
                        continue
                    if wanted & set(self.resident):
                        if inline:                          # let this round's solves run first
                            self.jobs.appendleft(key)
                            self.factoring.discard(key)
                            return 0
                        self._wake.wait(timeout=0.005)
                        continue
                    self._fail_key(key, MemoryError(f"system {key} does not fit in the HBM budget"))
                    self.factoring.discard(key)
                    return 0
            except Exception as e:                          # a library error: fail its requests
                with self._lock:
                    self._fail_key(key, e)
                    self.factoring.discard(key)
                return 0
            if self.factor_backend is not self.backend and hasattr(self.backend, "adopt"):
                self.backend.adopt(h)                       # its solves run on the solve stream
            with self._lock:
                nbytes = self.factor_backend.resident_bytes(h)
                self.resident[key] = _Resident(h, nbytes, time.perf_counter())
                self.n_factored += 1
                waiters = self.factor_waiters.pop(key, [])
                for req in waiters:
                    self._complete_factor(req, nbytes)
                self.factoring.discard(key)
                self._wake.notify_all()
                return len(waiters)

    # ------------------------------------------------------------ solve rounds
    def _ws_bytes(self, n, width) -> int:
        """Device bytes of the GMRES workspace of one system at a width: Krylov
        basis and preconditioned vectors (2 m + 1 vectors), five more vectors and
        the extended vector of the solve (at most 2 n rows)."""
        m = self.restart if self.cycle is None else self.cycle
        return int((2 * m + 1 + 5 + 2) * n * width * 8)

    def _make_room(self, keep, need) -> None:
        """Lock held: frees device memory so that the resident footprint plus
        `need` fits the budget: trims the workspaces of idle handles, then evicts
        idle systems (least recently used first).  Systems in `keep` stay."""
        if self._resident_bytes() + need <= self.budget:
            return
        trim = getattr(self.backend, "trim", None)
        if trim is not None:
            for k, r in self.resident.items():
                if k in keep or k in self.busy:
                    continue
                trim(r.handle)
                r.bytes = self.backend.resident_bytes(r.handle)
        wanted = keep | self.busy | {q.key for q in self.pending}
        while self._resident_bytes() + need > self.budget:
            idle = [k for k in self.resident if k not in wanted]
            if not idle:
                idle = [k for k in self.resident if k not in keep and k not in self.busy]
            if not idle:
                return
            self._evict(idle[0])

    def _solve_ready(self) -> int:
        with self._lock:
            groups: "collections.OrderedDict[str, list]" = collections.OrderedDict()
            width: dict[str, int] = {}
            rest = collections.deque()
            for req in self.pending:
                if req.future.cancelled():          # cancelled while queued: dropped
                    continue
                if req.x is None:                   # first round of this request
                    k = req.cols()
                    req.x = np.zeros((req.b.shape[0], k))
                    req.its = np.zeros(k, dtype=np.int64)
                    req.rr = np.full(k, np.inf)
                    req.conv = np.zeros(k, dtype=bool)
                cols = [c for c in range(req.cols()) if not req.conv[c]]
                k = len(cols)
                if req.key not in self.resident or req.key in self.busy:
                    rest.append(req)
                    continue
                if req.key not in groups and len(groups) >= self.max_batch_systems:
                    rest.append(req)
                    continue
                if width.get(req.key, 0) + k > self.max_width:
                    rest.append(req)
                    continue
                groups.setdefault(req.key, []).append((req, cols))
                width[req.key] = width.get(req.key, 0) + k
            self.pending = rest
            if not groups:
                return 0
            self.busy |= set(groups)
            handles = {key: self.resident[key].handle for key in groups}
            ns = {key: self.specs[key].n for key in groups}
            pw = {}
            for key in groups:
                w = 1
                while w < width[key]:
                    w *= 2
                pw[key] = w
            self._make_room(set(groups), sum(self._ws_bytes(ns[k], pw[k]) for k in groups))
        # one batched call per width class
        classes: dict[int, list] = {}
        for key in groups:
            classes.setdefault(pw[key], []).append(key)
        x0 = self.cycle is not None
        restart = self.restart if self.cycle is None else self.cycle
        maxit = self.maxit if self.cycle is None else self.cycle
        results = {}
        try:
            for wcls in sorted(classes):
                items, spans = [], []
                for key in classes[wcls]:
                    n = ns[key]
                    B = np.zeros((n, wcls))
                    X0 = np.zeros((n, wcls))
                    c0 = 0
                    for req, cols in groups[key]:
                        bb = req.b.reshape(n, -1)
                        for c in cols:
                            B[:, c0] = bb[:, c]
                            X0[:, c0] = req.x[:, c]
                            c0 += 1
                    items.append((handles[key], B, X0))
                for attempt in (0, 1):
                    try:
                        out = self.backend.solve_batch(items, wcls, self.tol, restart, maxit, x0=x0)
                        break
                    except OutOfBudget:
                        if attempt:
                            raise
                        with self._lock:            # evict the idle systems and retry once
                            wanted = set(groups) | self.busy
                            for k in [k for k in self.resident if k not in wanted]:
                                self._evict(k)
                for key, res in zip(classes[wcls], out):
                    results[key] = res
        except Exception as e:
            with self._lock:
                self.busy -= set(groups)
                for key in groups:
                    for req, _ in groups[key]:
                        if not req.future.cancelled():
                            req.future.set_exception(e)
                self._wake.notify_all()
            return 0
        now = time.perf_counter()
        done = 0
        with self._lock:
            self.busy -= set(groups)
            again = []
            for key in groups:
                X, its, rr = results[key]
                if key in self.resident:
                    r = self.resident[key]
                    r.last_use = now
                    r.bytes = self.backend.resident_bytes(r.handle)
                    self.resident.move_to_end(key)
                c0 = 0
                for req, cols in groups[key]:
                    for c in cols:
                        req.x[:, c] = X[:, c0]
                        req.its[c] += int(its[c0])
                        req.rr[c] = float(rr[c0])
                        req.conv[c] = req.rr[c] <= self.tol
                        c0 += 1
                    finished = all(req.conv[c] or req.its[c] >= self.maxit for c in range(req.cols()))
                    if req.future.cancelled():      # cancelled during the round: dropped
                        continue
                    if self.cycle is None or finished:
                        x = req.x[:, 0] if req.b.ndim == 1 else req.x.copy()
                        req.future.set_result((x, req.its.astype(np.int32), req.rr.copy()))
                        self.latencies["solve"].append(now - req.arrival)
                        done += 1
                    else:
                        again.append(req)
            # unfinished requests keep their place ahead of later arrivals
            self.pending.extendleft(reversed(again))
            self.n_solved += done
            self.batches.append(len(groups))
            self.n_rounds += 1
            self._wake.notify_all()
        return done
