"""ctypes binding of liblorax.so (argument marshalling only).

Every numerical step runs in the library's HIP kernels; this module converts
NumPy arrays / torch tensors to plain pointers and sizes and raises LoraxError
on a non-zero status.  Importing it loads liblorax.so and fails loudly when the
library has not been built.
"""
from __future__ import annotations

import ctypes as C
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "liblorax.so")

LRX_OK, LRX_EINVAL, LRX_ENOMEM, LRX_ESINGULAR, LRX_ENOCONV, LRX_EDEVICE, LRX_EBUSY = range(7)
STATUS_NAMES = {0: "LRX_OK", 1: "LRX_EINVAL", 2: "LRX_ENOMEM", 3: "LRX_ESINGULAR",
                4: "LRX_ENOCONV", 5: "LRX_EDEVICE", 6: "LRX_EBUSY"}
LRX_FP64, LRX_MIXED, LRX_MIXED_BF16 = 0, 1, 2
LRX_COLORED, LRX_NATURAL = 0, 1
ORDERS = {"colored": LRX_COLORED, "natural": LRX_NATURAL}
LRX_SVD, LRX_RRQR, LRX_RAND = 0, 1, 2
COMPRESS = {"svd": LRX_SVD, "rrqr": LRX_RRQR, "rand": LRX_RAND}
PRECISION = {"fp64": LRX_FP64, "mixed": LRX_MIXED, "mixed_bf16": LRX_MIXED_BF16}
RULES = {"cutoff1": 0, "frob": 1}


class LoraxError(RuntimeError):
    def __init__(self, status, msg):
        super().__init__(f"{STATUS_NAMES.get(status, status)}: {msg}")
        self.status = status


class Csr(C.Structure):
    _fields_ = [("n", C.c_int32), ("nnz", C.c_int64), ("row_ptr", C.POINTER(C.c_int64)),
                ("col_idx", C.POINTER(C.c_int32)), ("val", C.POINTER(C.c_double))]


class Tree(C.Structure):
    _fields_ = [("depth", C.c_int32), ("perm", C.POINTER(C.c_int32)),
                ("leaf_ptr", C.POINTER(C.c_int32))]


class Opts(C.Structure):
    _fields_ = [("epsilon", C.c_double), ("precision", C.c_int32), ("compress", C.c_int32),
                ("order", C.c_int32), ("hbm_budget_bytes", C.c_int64), ("stream", C.c_void_p),
                ("rule", C.c_int32), ("symmetric", C.c_int32)]


class Stats(C.Structure):
    _fields_ = [("depth", C.c_int32), ("n_compressions", C.c_int32),
                ("n_colour_steps", C.c_int32), ("max_rank", C.c_int32),
                ("mean_rank", C.c_double), ("rank_max_by_level", C.c_int32 * 32),
                ("rank_mean_by_level", C.c_double * 32),
                ("mean_node_size_by_level", C.c_double * 32),
                ("extended_size", C.c_int64), ("max_compression_error", C.c_double),
                ("factor_bytes", C.c_int64),
                ("solve_bytes", C.c_int64), ("factor_flops", C.c_int64),
                ("t_plan_ms", C.c_double), ("t_factor_ms", C.c_double),
                ("t_sync_ms", C.c_double), ("t_solve_prog_ms", C.c_double),
                ("device_bytes", C.c_int64), ("flops_compress", C.c_double), ("flops_pivot", C.c_double),
                ("flops_schur", C.c_double), ("flops_project", C.c_double),
                ("level_norm_by_level", C.c_double * 32), ("sweep_stages", C.c_int64),
                ("sweep_launches", C.c_int64), ("t_host_compress_ms", C.c_double),
                ("t_host_node_ms", C.c_double)]


class KernelTime(C.Structure):
    _fields_ = [("launches", C.c_int64), ("total_ms", C.c_double), ("bytes", C.c_double),
                ("flops", C.c_double)]


class Timing(C.Structure):
    _fields_ = [("k", KernelTime * 8)]


KERNEL_CLASSES = {0: "compress", 1: "factor_node", 2: "solve_fwd", 3: "solve_bwd", 4: "spmv",
                  5: "schur", 6: "project", 7: "compress_gram"}


class PlanInfo(C.Structure):
    _fields_ = [("depth", C.c_int32), ("n_supernodes", C.c_int32),
                ("n_colour_steps", C.c_int32), ("colours_by_level", C.c_int32 * 32),
                ("n_candidates", C.c_int64), ("n_schur_pairs", C.c_int64),
                ("n_edges_created", C.c_int64), ("candidates_by_level", C.c_int64 * 32)]


class Tune(C.Structure):
    _fields_ = [("gemm_kc", C.c_int32), ("gemm_f64_valu", C.c_int32), ("sweep_nk_max", C.c_int32),
                ("compress_nt_small", C.c_int32), ("compress_nt_mid", C.c_int32), ("gemm_grid", C.c_int32),
                ("solve_graph", C.c_int32), ("compress_gram", C.c_int32), ("large_split_c", C.c_int32)]


TUNE_FIELDS = ("gemm_kc", "gemm_f64_valu", "sweep_nk_max", "compress_nt_small", "compress_nt_mid", "gemm_grid",
               "solve_graph", "compress_gram", "large_split_c")


# every symbol declared in include/lorax.h
EXPORTS = ("lrx_factor", "lrx_factor_dev", "lrx_factor_batch", "lrx_timing_enable", "lrx_timing_read", "lrx_solve", "lrx_solve_dev",
           "lrx_solve_batch_dev", "lrx_gmres", "lrx_gmres_dev", "lrx_gmres_batch_dev", "lrx_set_stream",
           "lrx_free", "lrx_stats", "lrx_ranks", "lrx_compression_tails", "lrx_compression_shape", "lrx_gmres_history", "lrx_plan_inspect",
           "lrx_last_error", "lrx_version", "lrx_tune_get", "lrx_tune_set",
           "lrx_solve_dev_noalloc", "lrx_gmres_batch_dev_x0", "lrx_trim")


def _load():
    if not os.path.exists(LIB_PATH):
        raise ImportError(f"{LIB_PATH} is not built: run __graft_entry__.build() "
                          "or python -m paper_1510_07363_amd.build")
    lib = C.CDLL(LIB_PATH)
    P = C.POINTER
    i32p, f64p = P(C.c_int32), P(C.c_double)
    sig = {
        "lrx_factor": (C.c_int, [P(Csr), P(Tree), P(Opts), P(C.c_void_p)]),
        "lrx_factor_dev": (C.c_int, [P(Csr), C.c_void_p, P(Tree), P(Opts), P(C.c_void_p)]),
        "lrx_factor_batch": (C.c_int, [C.c_int32, P(Csr), P(C.c_void_p), P(Tree), P(Opts), P(C.c_void_p)]),
        "lrx_timing_enable": (None, [C.c_int32]),
        "lrx_timing_read": (C.c_int, [P(Timing), C.c_int32]),
        "lrx_solve": (C.c_int, [C.c_void_p, C.c_int32, f64p, C.c_int64, f64p, C.c_int64]),
        "lrx_solve_dev": (C.c_int, [C.c_void_p, C.c_int32, C.c_void_p, C.c_void_p]),
        "lrx_solve_dev_noalloc": (C.c_int, [C.c_void_p, C.c_int32, C.c_void_p, C.c_void_p]),
        "lrx_solve_batch_dev": (C.c_int, [C.c_int32, P(C.c_void_p), C.c_int32, P(C.c_void_p),
                                          P(C.c_void_p)]),
        "lrx_gmres": (C.c_int, [P(Csr), C.c_void_p, C.c_int32, f64p, f64p, C.c_double,
                                C.c_int32, C.c_int32, i32p, f64p]),
        "lrx_gmres_dev": (C.c_int, [C.c_void_p, C.c_int32, C.c_void_p, C.c_void_p, C.c_double,
                                    C.c_int32, C.c_int32, i32p, f64p]),
        "lrx_gmres_batch_dev": (C.c_int, [C.c_int32, P(C.c_void_p), C.c_int32, P(C.c_void_p),
                                          P(C.c_void_p), C.c_double, C.c_int32, C.c_int32, i32p, f64p]),
        "lrx_gmres_batch_dev_x0": (C.c_int, [C.c_int32, P(C.c_void_p), C.c_int32, P(C.c_void_p),
                                             P(C.c_void_p), C.c_double, C.c_int32, C.c_int32, i32p, f64p]),
        "lrx_set_stream": (C.c_int, [C.c_void_p, C.c_void_p]),
        "lrx_trim": (C.c_int, [C.c_void_p]),
        "lrx_free": (C.c_int, [C.c_void_p]),
        "lrx_stats": (C.c_int, [C.c_void_p, P(Stats)]),
        "lrx_ranks": (C.c_int, [C.c_void_p, i32p, i32p, i32p]),
        "lrx_compression_tails": (C.c_int, [C.c_void_p, C.c_int32, f64p, C.c_int32, i32p]),
        "lrx_compression_shape": (C.c_int, [C.c_void_p, C.c_int32, i32p, i32p]),
        "lrx_gmres_history": (C.c_int, [C.c_void_p, C.c_int32, f64p, C.c_int32, i32p]),
        "lrx_plan_inspect": (C.c_int, [P(Csr), P(Tree), C.c_int32, P(PlanInfo)]),
        "lrx_last_error": (C.c_char_p, []),
        "lrx_version": (C.c_char_p, []),
        "lrx_tune_get": (C.c_int, [P(Tune)]),
        "lrx_tune_set": (C.c_int, [P(Tune)]),
    }
    for name, (res, args) in sig.items():
        f = getattr(lib, name)
        f.restype = res
        f.argtypes = args
    return lib


_lib = _load()


def _check(status):
    if status != LRX_OK:
        raise LoraxError(status, _lib.lrx_last_error().decode())


def version():
    return _lib.lrx_version().decode()


def _ptr(a, ctype):
    return a.ctypes.data_as(C.POINTER(ctype))


class _CsrArgs:
    """Holds contiguous copies of the CSR arrays while a call runs."""

    def __init__(self, row_ptr, col_idx, val):
        self.rp = np.ascontiguousarray(row_ptr, dtype=np.int64)
        self.ci = np.ascontiguousarray(col_idx, dtype=np.int32)
        self.v = np.ascontiguousarray(val, dtype=np.float64)
        self.s = Csr(len(self.rp) - 1, int(self.rp[-1]), _ptr(self.rp, C.c_int64),
                     _ptr(self.ci, C.c_int32), _ptr(self.v, C.c_double))


class _TreeArgs:
    def __init__(self, perm, leaf_ptr, depth):
        self.perm = np.ascontiguousarray(perm, dtype=np.int32)
        self.lp = np.ascontiguousarray(leaf_ptr, dtype=np.int32)
        self.s = Tree(int(depth), _ptr(self.perm, C.c_int32), _ptr(self.lp, C.c_int32))


def tune_get():
    """Current launch shapes of the hot kernels (lrx_tune_get) as a dict."""
    t = Tune()
    _check(_lib.lrx_tune_get(C.byref(t)))
    return {f: int(getattr(t, f)) for f in TUNE_FIELDS}


def tune_set(**fields):
    """Sets some launch shapes (lrx_tune_set); the others keep their values."""
    cur = tune_get()
    for k, v in fields.items():
        if k not in TUNE_FIELDS:
            raise KeyError(k)
        cur[k] = int(v)
    t = Tune(*[cur[f] for f in TUNE_FIELDS])
    _check(_lib.lrx_tune_set(C.byref(t)))


def timing_enable(classes=None):
    """Record HIP events around the launches of the given kernel classes (names
    of KERNEL_CLASSES; None = all, [] = off)."""
    if classes is None:
        mask = 0xFF
    else:
        inv = {v: k for k, v in KERNEL_CLASSES.items()}
        mask = 0
        for c in classes:
            mask |= 1 << inv[c]
    _lib.lrx_timing_enable(mask)


def timing_read(reset=True):
    """Per kernel class: launches, total_ms, bytes, flops (event-measured)."""
    t = Timing()
    _check(_lib.lrx_timing_read(C.byref(t), 1 if reset else 0))
    return {name: dict(launches=int(t.k[i].launches), total_ms=float(t.k[i].total_ms),
                       bytes=float(t.k[i].bytes), flops=float(t.k[i].flops))
            for i, name in KERNEL_CLASSES.items()}


def plan_inspect(row_ptr, col_idx, perm, leaf_ptr, depth, order="colored"):
    """Host-only symbolic plan counts (no device call)."""
    A = _CsrArgs(row_ptr, col_idx, np.zeros(len(col_idx)))
    T = _TreeArgs(perm, leaf_ptr, depth)
    info = PlanInfo()
    _check(_lib.lrx_plan_inspect(C.byref(A.s), C.byref(T.s), ORDERS[order], C.byref(info)))
    d = int(info.depth)
    return dict(depth=d, n_supernodes=int(info.n_supernodes),
                n_colour_steps=int(info.n_colour_steps),
                colours_by_level={i: int(info.colours_by_level[i]) for i in range(1, d + 1)},
                candidates_by_level={i: int(info.candidates_by_level[i]) for i in range(1, d + 1)},
                n_candidates=int(info.n_candidates), n_schur_pairs=int(info.n_schur_pairs),
                n_edges_created=int(info.n_edges_created))


def factor_batch(systems, epsilon, order="colored", compress="svd", stream=None, hbm_budget_bytes=0,
                 precision="fp64", val_dev=None, rule="cutoff1", symmetric=False):
    """Factorizes several systems in one lrx_factor_batch call.
    systems: sequence of (row_ptr, col_idx, val, perm, leaf_ptr, depth); with
    val_dev (a sequence of device addresses of each system's values) val may be None.
    Returns one Factor per system (each equal to factoring it alone)."""
    systems = list(systems)
    k = len(systems)
    As = [_CsrArgs(rp, ci, v if v is not None else np.zeros(0)) for rp, ci, v, _, _, _ in systems]
    Ts = [_TreeArgs(pm, lp, d) for _, _, _, pm, lp, d in systems]
    A_arr = (Csr * k)(*[a.s for a in As])
    T_arr = (Tree * k)(*[t.s for t in Ts])
    o = Opts(float(epsilon), PRECISION[precision], COMPRESS[compress], ORDERS[order],
             int(hbm_budget_bytes), C.c_void_p(stream) if stream else None, RULES[rule], int(symmetric))
    hs = (C.c_void_p * k)()
    vd = None if val_dev is None else (C.c_void_p * k)(*[int(v) for v in val_dev])
    _check(_lib.lrx_factor_batch(k, A_arr, vd, T_arr, C.byref(o), hs))
    return [Factor._adopt(C.c_void_p(hs[i]), As[i]) for i in range(k)]


class Factor:
    """A factorization resident in HBM (wraps lrx_handle)."""

    def __init__(self, row_ptr, col_idx, val, perm, leaf_ptr, depth, epsilon,
                 order="colored", compress="svd", stream=None, hbm_budget_bytes=0,
                 val_dev=None, precision="fp64", rule="cutoff1", symmetric=False):
        """val: host values, or None with val_dev = device address of the values.
        precision: "fp64" or "mixed" (FP32 compression arithmetic and FP32 stored
        factor for the solve; FP64 pivots, Schur updates and GMRES)."""
        if val is None:
            val = np.zeros(0)
        self._A = _CsrArgs(row_ptr, col_idx, val)
        T = _TreeArgs(perm, leaf_ptr, depth)
        o = Opts(float(epsilon), PRECISION[precision], COMPRESS[compress], ORDERS[order],
                 int(hbm_budget_bytes), C.c_void_p(stream) if stream else None, RULES[rule],
                 int(symmetric))
        h = C.c_void_p()
        if val_dev is not None:
            _check(_lib.lrx_factor_dev(C.byref(self._A.s), C.c_void_p(val_dev), C.byref(T.s),
                                       C.byref(o), C.byref(h)))
        else:
            _check(_lib.lrx_factor(C.byref(self._A.s), C.byref(T.s), C.byref(o), C.byref(h)))
        self._h = h
        self.n = len(self._A.rp) - 1

    @classmethod
    def _adopt(cls, h, A):
        F = cls.__new__(cls)
        F._A, F._h, F.n = A, h, len(A.rp) - 1
        return F

    # ------------------------------------------------------------ host arrays
    def solve(self, b):
        """x ~ A^{-1} b (Algorithms 2-4); b of shape (n,) or (n, nrhs)."""
        b = np.asarray(b, dtype=np.float64)
        vec = b.ndim == 1
        B = np.asfortranarray(b.reshape(self.n, -1))
        X = np.zeros_like(B, order="F")
        _check(_lib.lrx_solve(self._h, B.shape[1], _ptr(B, C.c_double), self.n,
                              _ptr(X, C.c_double), self.n))
        return X[:, 0] if vec else X

    def gmres(self, b, tol=1e-10, restart=30, maxit=500, raise_on_noconv=True, val=None):
        """Right-preconditioned GMRES; returns (x, iters, relres).  A is the
        matrix factored (its host values; pass val for a handle factored from
        device values); the library rejects a matrix that differs from the
        handle's resident copy."""
        A = self._A
        if val is not None:
            A = _CsrArgs(self._A.rp, self._A.ci, val)
        if len(A.v) != len(A.ci):
            raise ValueError("the handle was factored from device values: pass val")
        b = np.asarray(b, dtype=np.float64)
        vec = b.ndim == 1
        B = np.asfortranarray(b.reshape(self.n, -1))
        k = B.shape[1]
        X = np.zeros_like(B, order="F")
        its = np.zeros(k, dtype=np.int32)
        rr = np.zeros(k, dtype=np.float64)
        st = _lib.lrx_gmres(C.byref(A.s), self._h, k, _ptr(B, C.c_double),
                            _ptr(X, C.c_double), float(tol), int(restart), int(maxit),
                            _ptr(its, C.c_int32), _ptr(rr, C.c_double))
        if st != LRX_OK and (st != LRX_ENOCONV or raise_on_noconv):
            _check(st)
        return (X[:, 0] if vec else X), its, rr

    # ------------------------------------------------------- device pointers
    def solve_dev(self, b_ptr, x_ptr, nrhs):
        """b_ptr, x_ptr: device addresses of n x nrhs column-major FP64 arrays."""
        _check(_lib.lrx_solve_dev(self._h, int(nrhs), C.c_void_p(b_ptr), C.c_void_p(x_ptr)))

    def solve_dev_noalloc(self, b_ptr, x_ptr, nrhs):
        """solve_dev with the library's static device scratch (no allocation)."""
        _check(_lib.lrx_solve_dev_noalloc(self._h, int(nrhs), C.c_void_p(b_ptr), C.c_void_p(x_ptr)))

    def gmres_dev(self, b_ptr, x_ptr, nrhs, tol=1e-10, restart=30, maxit=500):
        its = np.zeros(nrhs, dtype=np.int32)
        rr = np.zeros(nrhs, dtype=np.float64)
        st = _lib.lrx_gmres_dev(self._h, int(nrhs), C.c_void_p(b_ptr), C.c_void_p(x_ptr),
                                float(tol), int(restart), int(maxit), _ptr(its, C.c_int32),
                                _ptr(rr, C.c_double))
        if st not in (LRX_OK, LRX_ENOCONV):
            _check(st)
        return its, rr, st

    # ------------------------------------------------------------ counters
    def stats(self):
        s = Stats()
        _check(_lib.lrx_stats(self._h, C.byref(s)))
        d = int(s.depth)
        return dict(depth=d, n_compressions=int(s.n_compressions),
                    n_colour_steps=int(s.n_colour_steps), max_rank=int(s.max_rank),
                    mean_rank=float(s.mean_rank),
                    rank_max_by_level={i: int(s.rank_max_by_level[i]) for i in range(1, d + 1)},
                    rank_mean_by_level={i: float(s.rank_mean_by_level[i]) for i in range(1, d + 1)},
                    mean_node_size_by_level={i: float(s.mean_node_size_by_level[i])
                                             for i in range(1, d + 1)},
                    extended_size=int(s.extended_size),
                    max_compression_error=float(s.max_compression_error),
                    factor_bytes=int(s.factor_bytes),
                    solve_bytes=int(s.solve_bytes), factor_flops=int(s.factor_flops),
                    t_plan_ms=float(s.t_plan_ms), t_factor_ms=float(s.t_factor_ms),
                    t_sync_ms=float(s.t_sync_ms), t_solve_prog_ms=float(s.t_solve_prog_ms),
                    device_bytes=int(s.device_bytes),
                    flops_by_op={"compress": float(s.flops_compress), "pivot": float(s.flops_pivot),
                                 "schur": float(s.flops_schur), "project": float(s.flops_project)},
                    level_norm_by_level={i: float(s.level_norm_by_level[i]) for i in range(1, d + 1)},
                    sweep_stages=int(s.sweep_stages), sweep_launches=int(s.sweep_launches),
                    t_host_compress_ms=float(s.t_host_compress_ms), t_host_node_ms=float(s.t_host_node_ms))

    def ranks(self):
        n = self.stats()["n_compressions"]
        r = np.zeros(max(n, 1), dtype=np.int32)
        lv = np.zeros_like(r)
        js = np.zeros_like(r)
        _check(_lib.lrx_ranks(self._h, _ptr(r, C.c_int32), _ptr(lv, C.c_int32), _ptr(js, C.c_int32)))
        return r[:n], lv[:n], js[:n]

    def tails(self, idx):
        """SVD: [sigma_0, sigma_0..sigma_{c-1}]; RRQR: [|R11|, ||R22||_F at k = 0..rank]."""
        n = C.c_int32()
        _check(_lib.lrx_compression_tails(self._h, int(idx), None, 0, C.byref(n)))
        out = np.zeros(max(n.value, 1))
        _check(_lib.lrx_compression_tails(self._h, int(idx), _ptr(out, C.c_double), n.value,
                                          C.byref(n)))
        return out[:n.value]

    def gmres_history(self, rhs=0):
        """Relative residuals of the last GMRES call for one right-hand side: the
        true one at each restart, then the estimate after each Arnoldi step."""
        n = C.c_int32()
        _check(_lib.lrx_gmres_history(self._h, int(rhs), None, 0, C.byref(n)))
        out = np.zeros(max(n.value, 1))
        _check(_lib.lrx_gmres_history(self._h, int(rhs), _ptr(out, C.c_double), n.value, C.byref(n)))
        return out[:n.value]

    def shape(self, idx):
        """(rows, cols) of the stacked block of compression idx (lrx_compression_shape)."""
        m, c = C.c_int32(), C.c_int32()
        _check(_lib.lrx_compression_shape(self._h, int(idx), C.byref(m), C.byref(c)))
        return int(m.value), int(c.value)

    def trim(self):
        """Releases the solve/GMRES workspaces (lrx_trim); the factor stays resident."""
        _check(_lib.lrx_trim(self._h))

    def set_stream(self, stream):
        """Later solves and GMRES calls run on this HIP stream (an int address, or None)."""
        _check(_lib.lrx_set_stream(self._h, C.c_void_p(stream) if stream else None))

    def free(self):
        if self._h is not None and self._h.value:
            _check(_lib.lrx_free(self._h))
        self._h = None

    def __del__(self):
        try:
            self.free()
        except Exception:
            pass


def solve_batch_dev(factors, nrhs, b_ptrs, x_ptrs):
    """lrx_solve_batch_dev: one solve per factor, all sweeps of one (level, colour)
    step in one launch; b_ptrs[i], x_ptrs[i] are device addresses (n_i x nrhs,
    column-major).  Synchronous."""
    k = len(factors)
    hs = (C.c_void_p * k)(*[f._h for f in factors])
    bs = (C.c_void_p * k)(*[C.c_void_p(int(b)) for b in b_ptrs])
    xs = (C.c_void_p * k)(*[C.c_void_p(int(x)) for x in x_ptrs])
    _check(_lib.lrx_solve_batch_dev(int(k), hs, int(nrhs), bs, xs))


def gmres_batch_dev(factors, nrhs, b_ptrs, x_ptrs, tol=1e-10, restart=30, maxit=500, x0=False):
    """lrx_gmres_batch_dev: FGMRES of every factor's system in lock-step.
    b_ptrs[i], x_ptrs[i]: device addresses of n_i x nrhs column-major FP64 arrays.
    x0: x_ptrs hold the initial guesses (lrx_gmres_batch_dev_x0).
    Returns (iters, relres, status), each array of shape (k, nrhs)."""
    k = len(factors)
    hs = (C.c_void_p * k)(*[f._h.value for f in factors])
    bp = (C.c_void_p * k)(*[int(p) for p in b_ptrs])
    xp = (C.c_void_p * k)(*[int(p) for p in x_ptrs])
    its = np.zeros((k, nrhs), dtype=np.int32)
    rr = np.zeros((k, nrhs), dtype=np.float64)
    fn = _lib.lrx_gmres_batch_dev_x0 if x0 else _lib.lrx_gmres_batch_dev
    st = fn(k, hs, int(nrhs), bp, xp, float(tol), int(restart), int(maxit), _ptr(its, C.c_int32),
            _ptr(rr, C.c_double))
    if st not in (LRX_OK, LRX_ENOCONV):
        _check(st)
    return its, rr, st
