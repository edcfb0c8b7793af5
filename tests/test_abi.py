"""CPU-only checks of the C ABI: the library loads, exports every function
include/bqs.h declares, and rejects bad arguments before touching a GPU."""

import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "bqs.h")


def declared_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(bqs_[a-z_]+)\s*\(", text)))


@pytest.fixture(scope="module")
def bqs():
    import paper_1604_06697_amd as bqs_mod

    return bqs_mod


def test_header_declares_the_boundary():
    names = declared_functions()
    for fn in ("bqs_sort", "bqs_sort_pairs", "bqs_sort_segments", "bqs_workspace_bytes",
               "bqs_ctx_create", "bqs_ctx_destroy", "bqs_ctx_set_stream",
               "bqs_ctx_set_workspace", "bqs_ctx_sync_status", "bqs_status_str"):
        assert fn in names


def test_library_exports_every_declared_symbol(bqs):
    lib = ctypes.CDLL(bqs.LIBRARY)
    missing = [fn for fn in declared_functions() if not hasattr(lib, fn)]
    assert not missing, missing
    assert sorted(bqs.EXPORTED) == declared_functions()


def test_status_strings(bqs):
    for code, text in bqs.STATUS.items():
        assert bqs.lib.bqs_status_str(code).decode() == text
    assert bqs.lib.bqs_status_str(99).decode() == "unknown status"
    assert bqs.lib.bqs_version() >= 100


def test_ctx_params_roundtrip(bqs):
    ctx = bqs.Context(small_cutoff=1024, sample_max=63, pivot_mode=3, tile_ept=32)
    assert ctx.get_param("small_cutoff") == 1024
    assert ctx.get_param("sample_max") == 63
    assert ctx.get_param("pivot_mode") == 3
    assert ctx.get_param("tile_ept") == 32
    with pytest.raises(bqs.BqsError):
        ctx.set_param("pivot_mode", 7)
    for mode in (0, 1, 3, 5, 23, 33, 35, 55):
        ctx.set_param("pivot_mode", mode)
        assert ctx.get_param("pivot_mode") == mode
    ctx.set_param("pivot_mode", 3)
    ctx.set_param("pivot_skew", 8)
    assert ctx.get_param("pivot_skew") == 8
    for bad in (1, 65):
        with pytest.raises(bqs.BqsError):
            ctx.set_param("pivot_skew", bad)
    ctx.set_param("pivot_skew", 0)
    assert ctx.get_param("check_nan") == 0
    ctx.set_param("check_nan", 1)
    assert ctx.get_param("check_nan") == 1
    for t in (0, 1, 2):
        ctx.set_param("timing", t)
        assert ctx.get_param("timing") == t
    with pytest.raises(bqs.BqsError):
        ctx.set_param("timing", 3)
    with pytest.raises(bqs.BqsError):
        ctx.set_param("tile_ept", 12)
    assert bqs.lib.bqs_ctx_set_param(ctx._h, 77, 1) == 1
    assert ctx.get_param("mode") == bqs.MODE_ASYNC  # the default: calls only enqueue
    ctx.set_param("mode", bqs.MODE_LEVELS)
    assert ctx.get_param("mode") == bqs.MODE_LEVELS
    ctx.set_param("mode", bqs.MODE_PERSISTENT)
    assert ctx.get_param("mode") == bqs.MODE_PERSISTENT
    with pytest.raises(bqs.BqsError):
        ctx.set_param("mode", 3)
    assert ctx.get_param("mode") == bqs.MODE_PERSISTENT


def test_persistent_mode_clamps_the_cutoff_in_the_workspace_size(bqs):
    # the persistent kernel sorts small segments of at most 4096 keys, so
    # its lists are sized for that cutoff
    n = 1 << 22
    lv = bqs.Context(small_cutoff=8192)
    ps = bqs.Context(small_cutoff=8192, mode=bqs.MODE_PERSISTENT)
    p4 = bqs.Context(small_cutoff=4096, mode=bqs.MODE_PERSISTENT)
    ws = bqs.lib.bqs_workspace_bytes
    assert ws(ps._h, n, bqs.I32, 0, 1) == ws(p4._h, n, bqs.I32, 0, 1) > ws(lv._h, n, bqs.I32, 0, 1)


def test_workspace_bytes(bqs):
    ws = bqs.lib.bqs_workspace_bytes
    n = 1 << 20
    keys4 = ws(None, n, bqs.I32, 0, 1)
    keys8 = ws(None, n, bqs.F64, 0, 1)
    pairs = ws(None, n, bqs.U64, 4, 1)
    # the double buffer dominates: one copy of the keys (and two of the payloads)
    assert 4 * n <= keys4 < 4 * n * 1.2
    assert 8 * n <= keys8 < 8 * n * 1.2
    assert (8 + 4 + 4) * n <= pairs < 16 * n * 1.2
    assert ws(None, n, 99, 0, 1) == 0
    assert ws(None, n, bqs.I32, 3, 1) == 0
    assert ws(None, -1, bqs.I32, 0, 1) == 0
    assert ws(None, n, bqs.I32, 0, 20000) > keys4


def test_argument_errors_need_no_gpu(bqs):
    L = bqs.lib
    h = ctypes.c_void_p()
    assert L.bqs_ctx_create(ctypes.byref(h)) == 0
    try:
        assert L.bqs_ctx_create(None) == 1
        assert L.bqs_sort(None, 10, bqs.I32, h) == 1          # null keys
        assert L.bqs_sort(ctypes.c_void_p(64), -1, bqs.I32, h) == 1
        assert L.bqs_sort(ctypes.c_void_p(64), 10, 42, h) == 2  # bad dtype
        assert L.bqs_sort(ctypes.c_void_p(64), 10, bqs.I32, None) == 1
        assert L.bqs_sort(ctypes.c_void_p(64), 1, bqs.I32, h) == 0   # trivial
        assert L.bqs_sort(ctypes.c_void_p(64), 10, bqs.I32, h) == 1  # no workspace
        assert L.bqs_sort_pairs(ctypes.c_void_p(64), ctypes.c_void_p(128), 10, bqs.I32, 2, h) == 2
        assert L.bqs_sort_pairs(ctypes.c_void_p(64), None, 10, bqs.I32, 4, h) == 1
        assert L.bqs_sort_segments(ctypes.c_void_p(64), None, 3, 10, bqs.I32, h) == 1
        assert L.bqs_sort_segments(ctypes.c_void_p(64), ctypes.c_void_p(64), 0, 10, bqs.I32, h) == 0
        # workspace overlapping the keys is rejected
        assert L.bqs_ctx_set_workspace(h, ctypes.c_void_p(1 << 20), 1 << 30) == 0
        assert L.bqs_sort(ctypes.c_void_p((1 << 20) + 4096), 1000, bqs.I32, h) == 1
        assert L.bqs_ctx_set_workspace(h, None, 16) == 1
        # the no-allocation entry point checks its arguments before any GPU call
        assert L.bqs_sort_noalloc(None, 10, bqs.I32, None, None) == 1
        assert L.bqs_sort_noalloc(ctypes.c_void_p(64), -5, bqs.I32, None, None) == 1
        assert L.bqs_sort_noalloc(ctypes.c_void_p(64), 10, 42, None, None) == 2
        assert L.bqs_sort_noalloc(ctypes.c_void_p(64), 1 << 24, bqs.I32, None, None) == 7
        assert L.bqs_sort_noalloc(ctypes.c_void_p(64), 8_200_000, bqs.F64, None, None) == 7
    finally:
        L.bqs_ctx_destroy(h)
    L.bqs_ctx_destroy(None)


def test_binding_rejects_cpu_tensors(bqs):
    import torch

    with pytest.raises(bqs.BqsError):
        bqs.sort(torch.zeros(10, dtype=torch.int32))
    with pytest.raises(bqs.BqsError):
        bqs.Context().sort(torch.zeros(10, dtype=torch.int16))


def test_inplace_workspace_is_a_fraction_of_the_double_buffer(bqs):
    """In-place levels keep one class bit per key instead of a copy of the
    keys and payloads: the workspace shrinks to a few percent."""
    ws = bqs.lib.bqs_workspace_bytes
    ctx = bqs.Context(inplace=1)
    assert ctx.get_param("inplace") == 1
    n = 1 << 24
    for dt, vb, copy in ((bqs.I32, 0, 4), (bqs.F64, 0, 8), (bqs.U64, 4, 16), (bqs.I32, 8, 20)):
        out = ws(None, n, dt, vb, 1)
        inp = ws(ctx._h, n, dt, vb, 1)
        assert out >= copy * n
        # class bits (n / 8 bytes, per 4096-key tile) plus lists and counts:
        # under a tenth of the double-buffered workspace
        assert n // 8 <= inp < 0.1 * out, (dt, vb, inp, out)
    # segments: lists grow with k, the class bits do not
    assert ws(ctx._h, n, bqs.I32, 0, 20000) > ws(ctx._h, n, bqs.I32, 0, 1)
    ctx.set_param("inplace", 0)
    assert ws(ctx._h, n, bqs.I32, 0, 1) == ws(None, n, bqs.I32, 0, 1)
