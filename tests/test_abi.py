"""Host-side checks of the C ABI library (no device call): it loads, exports
every function declared in include/lorax.h, and its symbolic plan of Algorithm
1 has the same structure as the oracle's."""
import ctypes
import os
import re

import numpy as np
import pytest

import oracle
from paper_1510_07363_amd import workloads as w

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _declared():
    src = open(os.path.join(ROOT, "include", "lorax.h")).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(lrx_[a-z0-9_]+)\s*\(", src)))


def test_library_exports_every_declared_symbol():
    from paper_1510_07363_amd import lorax
    lib = ctypes.CDLL(lorax.LIB_PATH)
    names = _declared()
    assert len(names) >= 10
    for name in names:
        assert hasattr(lib, name), name
    assert set(names) == set(lorax.EXPORTS)
    assert lorax.version().startswith("lorax")


def _oracle_structure(p, order):
    F = oracle.factor(p.row_ptr, p.col_idx, p.val, p.perm, p.leaf_ptr, p.depth, 1e-3,
                      order=order, check=False)
    cbl = {}
    for c in F.compressions:
        cbl[c.level] = cbl.get(c.level, 0) + len(c.candidates)
    pairs = sum(len(ev[1].fwd) * len(ev[1].bwd) for ev in F.events
                if ev[0] == "elim" and ev[1].size > 0)
    return F.level_colours, cbl, pairs


@pytest.mark.parametrize("order", ["colored", "natural"])
@pytest.mark.parametrize("name,size", [("poisson2d_32", None), ("varcoef2d_256", 64),
                                       ("convdiff3d_64", 16)])
def test_plan_structure_matches_oracle(name, size, order):
    from paper_1510_07363_amd import lorax
    p = w.make_config(name, size=size)
    info = lorax.plan_inspect(p.row_ptr, p.col_idx, p.perm, p.leaf_ptr, p.depth, order)
    colours, cbl, pairs = _oracle_structure(p, order)
    assert info["colours_by_level"] == colours
    assert info["candidates_by_level"] == cbl
    assert info["n_schur_pairs"] == pairs
    assert info["n_supernodes"] == (1 << p.depth) - 1


def test_plan_rejects_bad_input():
    from paper_1510_07363_amd import lorax
    p = w.make_config("poisson2d_32")
    bad = p.perm.copy()
    bad[0] = bad[1]
    with pytest.raises(lorax.LoraxError) as e:
        lorax.plan_inspect(p.row_ptr, p.col_idx, bad, p.leaf_ptr, p.depth)
    assert e.value.status == lorax.LRX_EINVAL
    ci = p.col_idx.copy()
    ci[[0, 1]] = ci[[1, 0]]                       # unsorted row
    with pytest.raises(lorax.LoraxError):
        lorax.plan_inspect(p.row_ptr, ci, p.perm, p.leaf_ptr, p.depth)
    lp = p.leaf_ptr.copy()
    lp[-1] = p.n + 1                              # leaves do not cover exactly n rows
    with pytest.raises(lorax.LoraxError):
        lorax.plan_inspect(p.row_ptr, p.col_idx, p.perm, lp, p.depth)
    with pytest.raises(lorax.LoraxError):         # 2^depth > n
        lorax.plan_inspect(p.row_ptr, p.col_idx, p.perm, np.arange(2049, dtype=np.int32), 11)
    lp = p.leaf_ptr.copy()
    lp[3] = lp[2]                                 # empty leaf
    with pytest.raises(lorax.LoraxError):
        lorax.plan_inspect(p.row_ptr, p.col_idx, p.perm, lp, p.depth)


def test_factor_without_device_fails_cleanly():
    """On a host without a GPU the factor call reports an error status instead
    of falling back to anything."""
    import torch
    if torch.cuda.is_available():
        pytest.skip("a GPU is present")
    from paper_1510_07363_amd import lorax
    p = w.make_config("poisson2d_32")
    with pytest.raises(lorax.LoraxError) as e:
        lorax.Factor(p.row_ptr, p.col_idx, p.val, p.perm, p.leaf_ptr, p.depth, 1e-8)
    assert e.value.status in (lorax.LRX_EDEVICE, lorax.LRX_ENOMEM)


def test_factor_rejects_nonfinite_and_eps():
    from paper_1510_07363_amd import lorax
    p = w.make_config("poisson2d_32")
    v = p.val.copy()
    v[5] = np.nan
    with pytest.raises(lorax.LoraxError) as e:
        lorax.Factor(p.row_ptr, p.col_idx, v, p.perm, p.leaf_ptr, p.depth, 1e-8)
    assert e.value.status == lorax.LRX_EINVAL
    with pytest.raises(lorax.LoraxError) as e:
        lorax.Factor(p.row_ptr, p.col_idx, p.val, p.perm, p.leaf_ptr, p.depth, 1.5)
    assert e.value.status == lorax.LRX_EINVAL


def test_tune_table_validation():
    """lrx_tune_set accepts the documented ranges and rejects the rest (host only)."""
    from paper_1510_07363_amd import lorax
    base = lorax.tune_get()
    assert base["gemm_kc"] % 16 == 0 and base["sweep_nk_max"] in (1, 2, 4)
    try:
        lorax.tune_set(gemm_kc=64, sweep_nk_max=4, gemm_f64_valu=1, compress_nt_small=256, compress_nt_mid=512,
                       gemm_grid=1024, solve_graph=0, compress_gram=0, large_split_c=65)
        assert lorax.tune_get() == {"gemm_kc": 64, "gemm_f64_valu": 1, "sweep_nk_max": 4,
                                    "compress_nt_small": 256, "compress_nt_mid": 512, "gemm_grid": 1024,
                                    "solve_graph": 0, "compress_gram": 0, "large_split_c": 65}
        for bad in ({"gemm_kc": 24}, {"gemm_kc": 512}, {"sweep_nk_max": 3}, {"sweep_nk_max": 8}, {"gemm_f64_valu": 2},
                    {"compress_nt_small": 128}, {"compress_nt_mid": 2048}, {"gemm_grid": -1},
                    {"solve_graph": 2}, {"compress_gram": 3}, {"compress_gram": -1}, {"large_split_c": 64},
                    {"large_split_c": 65537}):
            with pytest.raises(lorax.LoraxError) as e:
                lorax.tune_set(**bad)
            assert e.value.status == lorax.LRX_EINVAL
        assert lorax.tune_get()["gemm_kc"] == 64          # a rejected call changes nothing
    finally:
        lorax.tune_set(**base)
