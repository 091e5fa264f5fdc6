"""The C ABI: the library loads, exports every function the header declares, and
rejects invalid arguments before touching the GPU (runs without a GPU)."""

import ctypes
import os
import re

import pytest

import paper_1612_07875_amd as dmd
from paper_1612_07875_amd import binding

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "dmd_stream.h")


def header_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(dmd_\w+)\s*\(", text)))


def test_header_declares_the_core_calls():
    names = header_functions()
    for core in ("dmd_stream_create", "dmd_stream_push", "dmd_stream_eigs", "dmd_stream_modes",
                 "dmd_stream_push_csr", "dmd_stream_destroy", "dmd_last_error"):
        assert core in names


def test_library_exports_every_declared_symbol():
    lib = dmd.load()
    for name in header_functions():
        assert hasattr(lib, name), name
        assert name in binding.SIGNATURES or name in binding.STRING_FUNCS, name


def test_opts_struct_matches_header_layout():
    # 6 int32 + 2 double + warm_start, max_block, eig_solver, buildup + 4 int32 reserved
    assert ctypes.sizeof(binding.Opts) == 6 * 4 + 2 * 8 + 8 * 4
    lib = dmd.load()
    o = binding.Opts()
    assert lib.dmd_opts_init(ctypes.byref(o)) == 0
    assert o.auto_solve == 1 and o.max_sweeps == 40 and o.rcond < 0
    assert lib.dmd_opts_init(None) == dmd.E_INVAL


@pytest.mark.parametrize("n,m,r,msg", [
    (0, 8, 2, "n must be"),
    (100, 1, 1, "m must be"),
    (100, 300, 4, "m must be"),
    (100, 8, 0, "r must be"),
    (100, 8, 9, "r must be"),
    (100, 64, 33, "r must be"),
])
def test_create_rejects_bad_sizes_without_gpu(n, m, r, msg):
    lib = dmd.load()
    h = ctypes.c_void_p()
    rc = lib.dmd_stream_create(n, m, r, None, ctypes.byref(h))
    assert rc == dmd.E_INVAL
    assert msg in dmd.last_error()
    assert not h.value


def test_create_rejects_bad_options():
    lib = dmd.load()
    o = binding.Opts()
    lib.dmd_opts_init(ctypes.byref(o))
    o.reserved[3] = 1
    h = ctypes.c_void_p()
    assert lib.dmd_stream_create(100, 8, 2, ctypes.byref(o), ctypes.byref(h)) == dmd.E_INVAL
    lib.dmd_opts_init(ctypes.byref(o))
    o.dtype = 7
    assert lib.dmd_stream_create(100, 8, 2, ctypes.byref(o), ctypes.byref(h)) == dmd.E_INVAL
    assert lib.dmd_stream_create(100, 8, 2, None, None) == dmd.E_INVAL


def test_buildup_option_checks():
    """The build-up start: off by default, 0/1 only, dense single-push streams only."""
    lib = dmd.load()
    o = binding.Opts()
    lib.dmd_opts_init(ctypes.byref(o))
    assert o.buildup == 0
    h = ctypes.c_void_p()
    o.buildup = 2
    assert lib.dmd_stream_create(100, 8, 2, ctypes.byref(o), ctypes.byref(h)) == dmd.E_INVAL
    lib.dmd_opts_init(ctypes.byref(o))
    o.buildup = 1
    o.max_block = 4
    assert lib.dmd_stream_create(100, 8, 2, ctypes.byref(o), ctypes.byref(h)) == dmd.E_UNSUPPORTED
    lib.dmd_opts_init(ctypes.byref(o))
    o.buildup = 1
    o.dtype = binding.DTYPES["c64_csr"]
    assert lib.dmd_stream_create(100, 8, 2, ctypes.byref(o), ctypes.byref(h)) == dmd.E_UNSUPPORTED
    assert not h.value


def test_null_handle_calls_fail_cleanly():
    lib = dmd.load()
    assert lib.dmd_stream_push(None, None, None) == dmd.E_INVAL
    assert lib.dmd_stream_eigs(None, None, None, None, None) == dmd.E_INVAL
    assert lib.dmd_stream_modes(None, None, 0, None) == dmd.E_INVAL
    assert lib.dmd_stream_sync(None) == dmd.E_INVAL
    assert lib.dmd_stream_destroy(None) == dmd.OK
    assert "null handle" in dmd.last_error()


def test_version_string():
    assert b"gfx950" in dmd.load().dmd_version()


@pytest.mark.parametrize("dtype,max_block,code,msg", [
    (0, 65, dmd.E_INVAL, "max_block must be"),
    (0, -1, dmd.E_INVAL, "max_block must be"),
    (2, 2, dmd.E_UNSUPPORTED, "block pushes are for dense"),
])
def test_create_rejects_bad_block_options_without_gpu(dtype, max_block, code, msg):
    lib = dmd.load()
    o = binding.Opts()
    lib.dmd_opts_init(ctypes.byref(o))
    o.dtype = dtype
    o.max_block = max_block
    h = ctypes.c_void_p()
    rc = lib.dmd_stream_create(1000, 8, 4, ctypes.byref(o), ctypes.byref(h))
    assert rc == code
    assert msg in dmd.last_error()


@pytest.mark.parametrize("solver,warm,msg", [(3, 0, "unknown eig_solver"), (2, 1, "warm_start needs")])
def test_create_rejects_bad_solver_options_without_gpu(solver, warm, msg):
    lib = dmd.load()
    o = binding.Opts()
    lib.dmd_opts_init(ctypes.byref(o))
    o.eig_solver = solver
    o.warm_start = warm
    h = ctypes.c_void_p()
    assert lib.dmd_stream_create(1000, 8, 4, ctypes.byref(o), ctypes.byref(h)) == dmd.E_INVAL
    assert msg in dmd.last_error()


def test_footprint_is_host_only_and_adds_up_the_ring():
    """dmd_stream_footprint sizes a stream without a device: it grows with the
    ring (slots x roundup(n, 64) x element size) and checks like create."""
    n, m, r = 2_073_600, 64, 20
    ld = (n + 63) // 64 * 64
    f32 = dmd.footprint(n, m, r)
    f64 = dmd.footprint(n, m, r, dtype="f64")
    ring32 = (m + 2) * ld * 4
    assert ring32 < f32 < ring32 + 64 * 1024 * 1024
    # the FP64 ring is twice as large; workspaces grow by less than the ring
    assert f64 - f32 >= ring32
    # one more slot of n elements for every extra window column
    assert dmd.footprint(n, m + 1, r) - f32 >= ld * 4
    # a block stream keeps 2 max_block spare slots
    assert dmd.footprint(n, m, r, max_block=32) - f32 >= (2 * 32 - 1) * ld * 4
    sp = dmd.footprint(262144, 128, 24, dtype="c64_csr", max_nnz=2621)
    assert sp < 64 * 1024 * 1024
    lib = dmd.load()
    b = ctypes.c_int64(7)
    assert lib.dmd_stream_footprint(100, 8, 9, None, ctypes.byref(b)) == dmd.E_INVAL
    assert b.value == 0 and "r must be" in dmd.last_error()
    assert lib.dmd_stream_footprint(100, 8, 2, None, None) == dmd.E_INVAL
    with pytest.raises(dmd.DMDError):
        dmd.footprint(100, 300, 4)


def test_window_gram_rejects_bad_arguments_without_gpu():
    lib = dmd.load()
    g = ctypes.c_void_p(256)       # never dereferenced: every call below fails its checks
    assert lib.dmd_window_gram(None, 64, 64, 4, 0, 0, g, 4, None) == dmd.E_INVAL
    assert lib.dmd_window_gram(g, 64, 64, 0, 0, 0, g, 4, None) == dmd.E_INVAL
    assert lib.dmd_window_gram(g, 64, 64, 258, 0, 0, g, 300, None) == dmd.E_INVAL
    assert lib.dmd_window_gram(g, 63, 64, 4, 0, 0, g, 4, None) == dmd.E_INVAL
    assert lib.dmd_window_gram(g, 64, 64, 4, 2, 0, g, 4, None) == dmd.E_INVAL
    assert lib.dmd_window_gram(g, 64, 64, 4, 1, 2, g, 4, None) == dmd.E_UNSUPPORTED
    assert lib.dmd_window_gram(g, 65, 65, 4, 0, 0, g, 4, None) == dmd.E_INVAL   # column stride not 16 B
    assert "16-byte" in dmd.last_error()
