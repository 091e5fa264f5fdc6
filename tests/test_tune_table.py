"""The launch-shape tuning table on the host (no GPU): entries load from and
save to a text file, a malformed file is refused whole, lookups match a
stream shape by dtype, precision, n to within 1/8 octave, m, r and
max_block."""

import math

import pytest

import paper_1612_07875_amd as dmd


def nbucket(n):
    return round(8 * math.log2(n))


@pytest.fixture(autouse=True)
def _clean_table():
    dmd.tune_clear()
    yield
    dmd.tune_clear()


def write(path, lines):
    path.write_text("# comment\n" + "".join(l + "\n" for l in lines))


def test_load_lookup_save_roundtrip(tmp_path):
    n = 2_073_600
    f = tmp_path / "t.txt"
    # dtype precision nbucket m r max_block gram_iter proj_form gram_us step_us
    write(f, [f"0 0 {nbucket(n)} 64 20 32 2 2 91.5 4321.0", f"1 0 {nbucket(4096)} 32 10 1 1 0 3.0 0.0"])
    assert dmd.tune_lookup(n, 64, 20, max_block=32) is None
    dmd.tune_load(str(f))
    e = dmd.tune_lookup(n, 64, 20, max_block=32)
    assert e == {"gram_iter": 2, "proj_form": 2, "gram_us": 91.5, "step_us": 4321.0}
    # n within the same 1/8-octave bucket shares the entry; another bucket does not
    assert dmd.tune_lookup(n + 1000, 64, 20, max_block=32)["gram_iter"] == 2
    assert dmd.tune_lookup(int(n * 1.2), 64, 20, max_block=32) is None
    # every other key field must match
    assert dmd.tune_lookup(n, 64, 20) is None                      # max_block 1
    assert dmd.tune_lookup(n, 64, 21, max_block=32) is None
    assert dmd.tune_lookup(n, 63, 20, max_block=32) is None
    assert dmd.tune_lookup(n, 64, 20, max_block=32, precision="bf16x3") is None
    assert dmd.tune_lookup(4096, 32, 10, dtype="f64")["gram_iter"] == 1
    g = tmp_path / "saved.txt"
    dmd.tune_save(str(g))
    dmd.tune_clear()
    assert dmd.tune_lookup(n, 64, 20, max_block=32) is None
    dmd.tune_load(str(g))
    assert dmd.tune_lookup(n, 64, 20, max_block=32)["proj_form"] == 2
    # a later entry for the same key replaces the earlier one
    write(f, [f"0 0 {nbucket(n)} 64 20 32 4 1 88.0 4400.0"])
    dmd.tune_load(str(f))
    assert dmd.tune_lookup(n, 64, 20, max_block=32)["gram_iter"] == 4


@pytest.mark.parametrize("bad", ["0 0 160 64 20 32 3 0 1.0 0.0",      # slab form 3 does not exist
                                 "0 0 160 64 20 32 2 5 1.0 0.0",      # no projection form 5
                                 "0 0 160 64 20 32 2",                # truncated
                                 "tune me"])
def test_malformed_file_is_refused_whole(tmp_path, bad):
    f = tmp_path / "bad.txt"
    write(f, ["0 0 100 16 8 1 2 0 1.0 0.0", bad])
    with pytest.raises(dmd.DMDError) as ei:
        dmd.tune_load(str(f))
    assert ei.value.code == dmd.E_INVAL
    assert dmd.tune_lookup(2 ** 12.5, 16, 8) is None               # nothing of the file was taken


def test_missing_file_and_bad_arguments(tmp_path):
    with pytest.raises(dmd.DMDError):
        dmd.tune_load(str(tmp_path / "absent.txt"))
    lib = dmd.load()
    assert lib.dmd_tune_save(None) == dmd.E_INVAL
    assert lib.dmd_tune_lookup(100, 8, 4, None, None) == dmd.E_INVAL
    assert lib.dmd_tune(100, 8, 9, None, None, None) == dmd.E_INVAL


def test_cache_file_named_by_the_environment_is_loaded(tmp_path):
    import os
    import subprocess
    import sys
    f = tmp_path / "cache.txt"
    write(f, [f"0 0 {nbucket(300000)} 16 8 1 4 0 12.0 0.0"])
    root = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
    code = ("import paper_1612_07875_amd as d; e = d.tune_lookup(300000, 16, 8); "
            "print(e['gram_iter'] if e else 'none')")
    env = dict(os.environ, DMD_TUNE_CACHE=str(f))
    out = subprocess.run([sys.executable, "-c", code], cwd=root, env=env, capture_output=True, text=True,
                         timeout=120)
    assert out.returncode == 0, out.stderr
    assert out.stdout.strip().splitlines()[-1] == "4"
