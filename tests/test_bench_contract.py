"""The bench line's contract, checked on the CPU: one GPU only, and the roofline
entry computed from event-timed launches against MI355X's published peaks."""
import json
import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)
import bench  # noqa: E402


def test_more_than_one_gpu_is_refused():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"],
                       capture_output=True, text=True, timeout=120)
    assert r.returncode == 2
    msg = json.loads(r.stdout.strip().splitlines()[-1])
    assert "one GPU" in msg["error"] or "single-GPU" in msg["error"]


def test_published_peaks():
    assert bench.HBM_PEAK_GBS == 8000.0
    assert bench.FP64_PEAK_TFLOPS == 78.6
    assert bench.FP32_PEAK_TFLOPS == 157.3


def test_roofline_alu_and_hbm_entries():
    # 10 launches of 2 ms moving 8e9 bytes each: 4 TB/s, half the HBM peak
    t = {"solve_fwd": {"launches": 10, "total_ms": 20.0, "bytes": 8e10, "flops": 0.0}}
    r = bench.roofline(t, "solve_fwd")
    assert r["bound"] == "hbm" and r["unit"] == "GB/s"
    assert r["achieved"] == pytest.approx(4000.0)
    assert r["frac"] == pytest.approx(0.5)
    assert r["avg_launch_ms"] == pytest.approx(2.0) and r["launches"] == 10
    # 4 launches of 1 ms doing 78.6e9 flops each: the FP64 peak; in mixed
    # precision the compression is priced against the FP32 vector peak
    t = {"compress": {"launches": 4, "total_ms": 4.0, "bytes": 0.0, "flops": 4 * 78.6e9}}
    r = bench.roofline(t, "compress", "fp64")
    assert r["bound"] == "alu" and r["unit"] == "TFLOP/s"
    assert r["achieved"] == pytest.approx(78.6) and r["frac"] == pytest.approx(1.0)
    r = bench.roofline(t, "compress", "mixed")
    assert r["peak"] == 157.3 and r["frac"] == pytest.approx(78.6 / 157.3)
    t2 = {"factor_node": dict(t["compress"])}
    assert bench.roofline(t2, "factor_node", "mixed")["peak"] == 78.6


def test_roofline_mfma_classes():
    t = {"schur": {"launches": 2, "total_ms": 2.0, "bytes": 0.0, "flops": 2 * 78.6e9}}
    r = bench.roofline(t, "schur", "fp64")
    assert r["bound"] == "mfma" and r["peak"] == 78.6 and r["frac"] == pytest.approx(1.0)
    assert bench.roofline(t, "schur", "mixed")["peak"] == 157.3
    t = {"project": dict(t["schur"])}
    assert bench.roofline(t, "project", "mixed_bf16")["peak"] == 2500.0
