"""Launch-shape tuning on the GPU: dmd_tune measures the one-frame Gram
pass in each slab form and, for FP32 block streams, the pipelined block step
with one product per window, with window pairs (2r = 8 mod 16) and with one
banded product;
streams created afterwards take the recorded shapes.  Every shape the tuner
can choose must give oracle-correct results: the window-pair projection with
five column tiles (r = 20) is checked window by window here."""

import numpy as np
import pytest
import torch

import gen
from test_gpu_block import run_blocks

pytestmark = pytest.mark.gpu


def _dmd():
    import paper_1612_07875_amd as dmd
    return dmd


@pytest.fixture(autouse=True)
def _clean_table():
    dmd = _dmd()
    dmd.tune_clear()
    yield
    dmd.tune_clear()


def test_tune_gram_slab_form_is_recorded_and_used():
    dmd = _dmd()
    n, m, r = 300_001, 16, 8
    t = dmd.tune(n, m, r)
    assert t["gram_iter"] in (1, 2, 4) and t["gram_us"] > 0 and t["proj_form"] == 0
    assert dmd.tune_lookup(n, m, r) == t
    with dmd.Stream(n, m, r) as s:
        assert s.info().gram_iter == t["gram_iter"]
    with dmd.Stream(n, m, r, dtype="f64") as s:      # another key: the rule
        assert s.info().gram_iter in (1, 2, 4)
    t64 = dmd.tune(n, m, r, dtype="f64")
    with dmd.Stream(n, m, r, dtype="f64") as s:
        assert s.info().gram_iter == t64["gram_iter"]


def test_tune_block_projection_form():
    dmd = _dmd()
    n, m, r, kb = 131_072, 64, 20, 8
    t = dmd.tune(n, m, r, max_block=kb)
    assert t["proj_form"] in (1, 2, 3) and t["step_us"] > 0
    with dmd.Stream(n, m, r, max_block=kb) as s:
        assert s.info().proj_form == t["proj_form"]
    # no choice for split-BF16 projections; no pairs where 2r = 0 (mod 16)
    assert dmd.tune(n, m, r, max_block=kb, precision="bf16x3")["proj_form"] == 0
    assert dmd.tune(n, m, 16, max_block=kb)["proj_form"] in (1, 3)


@pytest.mark.parametrize("form", [1, 2, 3])
def test_block_projection_forms_match_the_oracle(tmp_path, form):
    """r = 20 (2r = 40: 48 of three tiles' columns per window, 80 of five
    tiles' per window pair, or 32-column tiles over all windows' columns, a
    tile touching at most two windows): every window of every block against
    the oracle, in the shape the tuning table names."""
    dmd = _dmd()
    H, W, m, r, kb = 120, 160, 64, 20, 8
    n = H * W
    nb = round(8 * np.log2(n))
    f = tmp_path / "t.txt"
    f.write_text(f"0 0 {nb} {m} {r} {kb} 1 {form} 0 0\n")
    dmd.tune_load(str(f))
    blocks = [8, 8, 8, 8, 8, 8, 8, 8, 8, 5, 8]
    frames = gen.BlobVideo(height=H, width=W, blob_sigma=6.0).frames(0, sum(blocks))
    X = torch.from_numpy(frames.T.copy()).cuda()
    with dmd.Stream(n, m, r, max_block=kb) as s:
        assert s.info().proj_form == form and s.info().gram_iter == 1
        run_blocks(s, X, frames, blocks, m, r, phi_tol=2e-4, every_window=True)
