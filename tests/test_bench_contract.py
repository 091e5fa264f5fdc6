"""The benchmark's contract on the host: one GPU only, and the roofline
arithmetic of its JSON line (bound, achieved, fraction) on hand-made kernel
timings."""

import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)
import bench  # noqa: E402


def test_more_than_one_gpu_is_refused():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"], cwd=ROOT,
                       capture_output=True, text=True, timeout=120)
    assert r.returncode == 2
    assert "one GPU" in r.stderr
    assert r.stdout.strip() == ""


def test_roofline_hbm_bound_kernel():
    kern = {"a": {"avg_us": 100.0}, "b": {"avg_us": 50.0}}
    out = bench.roofline_of(kern, {"a": 400e6, "b": 10e6}, {"a": "none.hip", "b": "none.hip"})
    assert out["kernel"] == "a" and out["bound"] == "hbm" and out["unit"] == "GB/s"
    assert out["achieved"] == pytest.approx(4000.0)
    assert out["frac"] == pytest.approx(0.5)
    assert out["floors_us"]["hbm"] == pytest.approx(50.0)
    assert kern["b"]["algorithmic_GBps"] == pytest.approx(200.0)


def test_roofline_mfma_bound_kernel():
    # 2 n m 2r k FP32 flops that need longer on the FP32 matrix peak than
    # their bytes need on HBM
    flops = 339.7e9
    kern = {"p": {"avg_us": 4320.0}}
    out = bench.roofline_of(kern, {"p": 11.4e9}, {"p": "none.hip"},
                            {"p": (flops, bench.FP32_MFMA_TFLOPS, "fp32")})
    assert out["bound"] == "mfma" and out["unit"] == "TFLOP/s" and out["peak"] == 157.3
    assert out["achieved"] == pytest.approx(flops / 4320e-6 / 1e12, rel=1e-3)
    assert out["frac"] == pytest.approx(out["achieved"] / 157.3, rel=1e-3)
    assert out["floors_us"]["mfma"] > out["floors_us"]["hbm"]


def test_gram_alone_rates():
    n, kb = 2073600, 32
    line = bench.gram_alone_line({"gram_columns": {"avg_us": 109.0}, "gram_block": {"avg_us": 390.0}}, n, kb)
    assert line["gram_columns"]["algorithmic_GBps"] == pytest.approx((bench.M + 2) * n * 4 / 109e-6 / 1e9, rel=1e-3)
    assert line["gram_block"]["algorithmic_GBps"] == pytest.approx((bench.M + 1 + 2 * kb) * n * 4 / 390e-6 / 1e9,
                                                                   rel=1e-3)
    assert "gram_block" not in bench.gram_alone_line({"gram_columns": {"avg_us": 109.0}}, n, None)


def test_cpu_baselines_report_cores_and_model():
    """Both CPU baselines (the SVD-route oracle per window, and the streaming
    method of snapshots per frame) on a small sample: positive rates, the
    threads used, the host's CPU count and model."""
    import numpy as np
    rng = np.random.default_rng(0)
    F = rng.standard_normal((12, 500))              # (frames, n)
    a = bench.cpu_baseline(F, 3, m=6, r=3)
    b = bench.cpu_baseline_streaming(F, 4, m=6, r=3)
    for x in (a, b):
        assert x["value"] > 0 and x["unit"] == "window updates/s" and x["kind"] == "oracle"
        assert x["cores"] >= 1 and x["nproc"] >= 1
        assert "n=500, m=6, r=3" in x["sample"]
    assert "streaming" in b["sample"]
