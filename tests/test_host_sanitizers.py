"""The host planner built with AddressSanitizer and UndefinedBehaviorSanitizer
(g++, host code only) on 2-D and 3-D problems: the same plan on one and on
four host threads, corrupted CSR and tree inputs refused with a message, and
no invalid memory access or undefined behaviour reported (the sanitizers abort
on the first one)."""
import os
import shutil
import subprocess

import numpy as np
import pytest

from paper_1510_07363_amd import workloads as w

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
CSRC = os.path.join(ROOT, "paper_1510_07363_amd", "csrc")


@pytest.fixture(scope="module")
def harness(tmp_path_factory):
    if shutil.which("g++") is None:
        pytest.skip("g++ not available")
    out = str(tmp_path_factory.mktemp("asan") / "plan_check")
    cmd = ["g++", "-std=c++17", "-O1", "-g", "-fno-omit-frame-pointer", "-fsanitize=address,undefined",
           "-fno-sanitize-recover=all", "-I", CSRC, os.path.join(ROOT, "tests", "host_plan_check.cpp"),
           os.path.join(CSRC, "plan.cpp"), "-o", out, "-lpthread"]
    subprocess.run(cmd, check=True, capture_output=True)
    return out


@pytest.mark.parametrize("name,size", [("poisson2d_32", None), ("varcoef2d_256", 96), ("convdiff3d_64", 20)])
def test_planner_under_sanitizers(harness, tmp_path, name, size):
    p = w.make_config(name, size=size)
    path = str(tmp_path / "prob.bin")
    with open(path, "wb") as f:
        np.array([p.n, p.row_ptr[-1], p.depth], dtype=np.int64).tofile(f)
        p.row_ptr.astype(np.int64).tofile(f)
        p.col_idx.astype(np.int32).tofile(f)
        p.perm.astype(np.int32).tofile(f)
        p.leaf_ptr.astype(np.int32).tofile(f)
    env = dict(os.environ, ASAN_OPTIONS="detect_leaks=1:abort_on_error=1", UBSAN_OPTIONS="print_stacktrace=1")
    r = subprocess.run([harness, path], capture_output=True, text=True, env=env, timeout=600)
    assert r.returncode == 0, (r.stdout[-2000:], r.stderr[-4000:])
    assert r.stdout.startswith("ok"), r.stdout
