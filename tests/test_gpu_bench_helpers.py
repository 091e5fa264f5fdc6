"""The benchmark's measurement helpers on the GPU: the background pass timed
alone and the one-frame Gram pass timed over back-to-back pushes report rates
that match their byte counts, and timing the background pass leaves the
stream's results unchanged."""

import os
import sys

import pytest
import torch

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)
import bench  # noqa: E402

pytestmark = pytest.mark.gpu


def test_background_alone_and_gram_back_to_back():
    import paper_1612_07875_amd as dmd
    n = 131072
    g = torch.Generator(device="cuda")
    g.manual_seed(11)
    frames = torch.rand((bench.M + 30, n), device="cuda", generator=g)
    s = dmd.Stream(n, bench.M, bench.R)
    try:
        for t in range(bench.M + 2):
            s.push(frames[t])
        fg0, bg0 = s.background()
        res = bench.background_alone(s, n, dmd, reps=3)
        fg1, bg1 = s.background()
        torch.cuda.synchronize()
    finally:
        s.close()
    assert res is not None and res["avg_us"] > 0
    assert res["algorithmic_bytes"] == (bench.M * 4 + 2 * 4) * n
    rate = res["algorithmic_bytes"] / (res["avg_us"] * 1e3)
    assert abs(res["algorithmic_GBps"] - rate) <= 1e-3 * rate + 0.1
    assert torch.equal(fg0, fg1) and torch.equal(bg0, bg1)

    gb = bench.gram_back_to_back(frames, n, dmd, reps=5)
    assert gb is not None and gb["launches"] == 5 and gb["avg_us"] > 0
    rate = (bench.M + 2) * n * 4 / (gb["avg_us"] * 1e3)
    assert abs(gb["algorithmic_GBps"] - rate) <= 1e-3 * rate + 0.1
    assert gb["frac_of_hbm_peak"] > 0
