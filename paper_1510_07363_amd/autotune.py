"""Autotuner of the library's launch shapes (lrx_tune_*), run on the device.

The tuned choices are those the library exposes in lrx_tune: the K chunk of the
matrix-core products (Schur updates and projection), the FP64 product engine
(MFMA or the VALU tile kernel), the grid of the products (a work-group per tile
or a persistent grid walking the tile list), the right-hand sides per
solve-sweep launch, and the threads per stacked block of the small-block
compression (two column ranges).  Every choice changes results only through rounding order.

Search: coordinate descent from the library defaults.  For each parameter in
turn, every candidate value is timed with the others fixed, and the fastest is
kept (ties: the earlier value).  A candidate's time is the median over
`repeats` of the event-timed kernel time of the phase it affects (lrx_timing_*):
the factorization kernels for the product and compression shapes, the solve
sweeps for the sweep width.  The first run of each shape is discarded (code
object load).  The winners go to a JSON cache, one entry per precision, with
the device and workload they were measured on; `load()` applies an entry with
lrx_tune_set.  Callers read the cache before
their timed region and never tune inside it.

Usage (on the GPU):
    python -m paper_1510_07363_amd.autotune --workload varcoef2d_256 \\
        --precision mixed --out paper_1510_07363_amd/tune_mi355x.json
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

import numpy as np

CANDIDATES = {
    "gemm_kc": [32, 64, 128, 256],
    "gemm_f64_valu": [0, 1],
    "compress_nt_small": [256, 512, 1024],
    "compress_nt_mid": [256, 512, 1024],
    "sweep_nk_max": [1, 2, 4],
    "gemm_grid": [0, 512, 1024, 2048],
}
FACTOR_CLASSES = ("compress", "compress_gram", "factor_node", "schur", "project")
SOLVE_CLASSES = ("solve_fwd", "solve_bwd")


def _phase_ms(lorax, p, precision, stream, val_dev, b_dev, x_dev, nrhs, classes):
    lorax.timing_enable(list(classes))
    lorax.timing_read(reset=True)
    F = lorax.Factor(p.row_ptr, p.col_idx, None, p.perm, p.leaf_ptr, p.depth, p.epsilon,
                     stream=stream, val_dev=val_dev, precision=precision)
    if any(c in SOLVE_CLASSES for c in classes):
        F.solve_dev(b_dev, x_dev, nrhs)
    F.free()
    t = lorax.timing_read(reset=True)
    lorax.timing_enable([])
    return sum(t[c]["total_ms"] for c in classes)


def tune(workload="varcoef2d_256", precision="mixed", repeats=3, size=None, log=print):
    import torch

    from . import lorax, workloads
    torch.cuda.set_device(0)
    p = workloads.make_config(workload, size=size)
    nrhs = p.rhs.shape[1]
    stream = torch.cuda.current_stream().cuda_stream
    val_d = torch.from_numpy(p.val).to("cuda:0")
    b_d = torch.from_numpy(np.ascontiguousarray(p.rhs.T)).to("cuda:0")
    x_d = torch.zeros_like(b_d)
    torch.cuda.synchronize()
    best = lorax.tune_get()
    history = []
    for name, values in CANDIDATES.items():
        if name == "gemm_f64_valu" and precision != "fp64":
            continue                         # the mixed products run FP32 on the matrix cores
        classes = SOLVE_CLASSES if name == "sweep_nk_max" else FACTOR_CLASSES
        times = {}
        for v in values:
            lorax.tune_set(**dict(best, **{name: v}))
            _phase_ms(lorax, p, precision, stream, val_d.data_ptr(), b_d.data_ptr(), x_d.data_ptr(), nrhs,
                      classes)                                   # first run: code objects
            ms = [_phase_ms(lorax, p, precision, stream, val_d.data_ptr(), b_d.data_ptr(), x_d.data_ptr(),
                            nrhs, classes) for _ in range(repeats)]
            times[v] = float(np.median(ms))
            history.append({"param": name, "value": v, "ms": times[v], "runs_ms": ms})
            log(f"[tune] {name}={v}: {times[v]:.3f} ms ({'+'.join(classes)})")
        pick = min(values, key=lambda v: (times[v], values.index(v)))
        best[name] = pick
        lorax.tune_set(**best)
        log(f"[tune] {name} -> {pick}")
    dev = torch.cuda.get_device_properties(0)
    return {"device": dev.name, "arch": getattr(dev, "gcnArchName", ""), "workload": workload,
            "size": size, "precision": precision, "repeats": repeats, "tune": best, "history": history,
            "date": time.strftime("%Y-%m-%d")}


def load(path, precision, lorax=None):
    """Applies the shapes tuned for `precision` in a cache file (lrx_tune_set);
    returns them, or None if the file or the entry does not exist."""
    if not os.path.exists(path):
        return None
    if lorax is None:
        from . import lorax
    with open(path) as f:
        d = json.load(f)
    entry = d.get(precision)
    if entry is None:
        return None
    lorax.tune_set(**entry["tune"])
    return entry["tune"]


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--workload", default="varcoef2d_256")
    ap.add_argument("--precision", default="mixed", choices=["fp64", "mixed"])
    ap.add_argument("--size", type=int, default=None)
    ap.add_argument("--repeats", type=int, default=3)
    ap.add_argument("--out", required=True)
    a = ap.parse_args()
    res = tune(a.workload, a.precision, a.repeats, a.size, log=lambda m: print(m, file=sys.stderr, flush=True))
    cache = {}
    if os.path.exists(a.out):
        with open(a.out) as f:
            cache = json.load(f)
    cache[a.precision] = res                 # one entry per precision
    with open(a.out, "w") as f:
        json.dump(cache, f, indent=1)
    print(json.dumps(res["tune"]))


if __name__ == "__main__":
    main()
