"""The C-ABI library loads on the host and exports every entry point that
include/gs.h declares; argument errors are reported on the host before any
GPU work (no compute calls here)."""
import ctypes
import re
import os

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def declared():
    src = open(os.path.join(ROOT, "include", "gs.h")).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(gs_[a-z_0-9]+)\s*\(", src)))


@pytest.fixture(scope="module")
def L():
    from paper_2407_00435_amd import build, binding
    if not os.path.exists(binding.lib_path):
        build.build()
    return binding


def test_every_declared_symbol_is_exported(L):
    lib = ctypes.CDLL(L.lib_path)
    names = declared()
    assert len(names) >= 15
    for n in names:
        assert hasattr(lib, n), n
    assert set(names) == set(L.EXPORTED), set(names) ^ set(L.EXPORTED)


def test_version_and_host_errors(L):
    lib = L.lib()
    assert lib.gs_version() == 2
    cams = (L.GsCamera * 1)()
    cams[0].width, cams[0].height, cams[0].fx, cams[0].fy = 64, 48, 50.0, 50.0
    nt, npx = ctypes.c_int64(), ctypes.c_int64()
    assert lib.gs_tile_count(ctypes.cast(cams, L._PC), 1, 16, ctypes.byref(nt), ctypes.byref(npx)) == 0
    assert (nt.value, npx.value) == (4 * 3, 64 * 48)
    # unsupported tile size
    assert lib.gs_tile_count(ctypes.cast(cams, L._PC), 1, 12, ctypes.byref(nt), ctypes.byref(npx)) == L.GS_ERR_UNSUPPORTED
    assert b"tile size" in lib.gs_last_error()
    # NULL scene, bad SH degree
    assert lib.gs_project(None, ctypes.cast(cams, L._PC), None, 1, 16, None, None, None) == L.GS_ERR_INVALID
    sc = L.GsScene()
    sc.n, sc.sh_degree = 10, 4
    assert lib.gs_project(ctypes.byref(sc), ctypes.cast(cams, L._PC), ctypes.c_void_p(1), 1, 16, None, None,
                          None) == L.GS_ERR_UNSUPPORTED
    # bad camera
    cams[0].fx = -1.0
    assert lib.gs_tile_count(ctypes.cast(cams, L._PC), 1, 16, ctypes.byref(nt), ctypes.byref(npx)) == L.GS_ERR_INVALID
    # workspace too small is a capacity error, found before any launch
    cams[0].fx = 50.0
    assert lib.gs_bin_sort(ctypes.c_void_p(256), 10, ctypes.cast(cams, L._PC), ctypes.c_void_p(256), 1, 16,
                           None, None, ctypes.c_void_p(256), None, 100, ctypes.c_void_p(256), None,
                           ctypes.c_void_p(256), ctypes.c_void_p(256), 16, None) == L.GS_ERR_CAPACITY
    assert b"workspace too small" in lib.gs_last_error()
    # sort: bad bit count
    assert lib.gs_sort_pairs(None, None, None, None, 10, 40, None, 0, None) == L.GS_ERR_INVALID
    assert lib.gs_set_tuning(b"radix_part", 1000) == L.GS_ERR_INVALID
    assert lib.gs_set_tuning(b"no_such_knob", 1) == L.GS_ERR_INVALID
    assert lib.gs_set_tuning(b"coarse_packed", 2) == L.GS_ERR_INVALID
    assert lib.gs_set_tuning(b"coarse_packed", 1) == 0


def test_package_fails_loudly_without_library(tmp_path, monkeypatch):
    from paper_2407_00435_amd import binding
    monkeypatch.setattr(binding, "lib_path", str(tmp_path / "missing.so"))
    monkeypatch.setattr(binding, "_lib", None)
    with pytest.raises(RuntimeError, match="missing"):
        binding.lib()


def test_contexts_hold_their_own_tuning(L):
    raw = L.raw_lib()
    h = ctypes.c_void_p()
    assert raw.gs_create(None, 0) == L.GS_ERR_INVALID
    assert raw.gs_create(ctypes.byref(h), -1) == L.GS_ERR_INVALID
    assert not h.value
    a, b = L.Context(0), L.Context(0)
    a.set_tuning("radix_part", 4096)
    b.set_tuning("radix_part", 16384)
    a.set_tuning("coarse_packed", 0)
    assert (a.get_tuning("radix_part"), b.get_tuning("radix_part")) == (4096, 16384)
    assert (a.get_tuning("coarse_packed"), b.get_tuning("coarse_packed")) == (0, 1)
    for k, v in (("raster_queue", 0), ("raster_grab", 1), ("raster_heavy", 0), ("raster_split", 0)):
        assert b.get_tuning(k) == v
    with pytest.raises(L.GsError, match="unknown tuning knob"):
        a.get_tuning("no_such_knob")
    with pytest.raises(L.GsError, match="radix_part"):
        a.set_tuning("radix_part", 1000)
    assert a.get_tuning("radix_part") == 4096  # a rejected value leaves the setting
    # the thread's current context follows `with`
    with b:
        assert L.context() is b and L.gs_get_tuning("radix_part") == 16384
        with a:
            assert L.context() is a
        assert L.context() is b
    assert L.context() is not a and L.context() is not b
    # workspace sizes depend on the context's tuning (the work queue)
    cams = (L.GsCamera * 1)()
    cams[0].width, cams[0].height, cams[0].fx, cams[0].fy = 640, 480, 500.0, 500.0
    pc = ctypes.cast(cams, L._PC)
    base = raw.gs_workspace_bytes(a.handle, pc, 1, 1000, 16, 100000)
    a.set_tuning("raster_queue", 1)
    assert raw.gs_workspace_bytes(a.handle, pc, 1, 1000, 16, 100000) > base
    assert raw.gs_workspace_bytes(None, pc, 1, 1000, 16, 100000) == 0
    a.close()
    b.close()


def test_calls_check_the_context_first(L):
    raw = L.raw_lib()
    cams = (L.GsCamera * 1)()
    cams[0].width, cams[0].height, cams[0].fx, cams[0].fy = 64, 48, 50.0, 50.0
    sc = L.GsScene()
    sc.n, sc.sh_degree = 10, 0
    assert raw.gs_project(None, ctypes.byref(sc), ctypes.cast(cams, L._PC), ctypes.c_void_p(256), 1, 16,
                          ctypes.c_void_p(256), None, None) == L.GS_ERR_INVALID
    assert b"context is NULL" in raw.gs_last_error()
    assert raw.gs_set_tuning(None, b"radix_part", 8192) == L.GS_ERR_INVALID
    assert raw.gs_l1_grad(None, None, None, 0, ctypes.c_float(1.0), None, ctypes.c_void_p(256), 1,
                          None) == L.GS_ERR_INVALID
    st, req = ctypes.c_int(), ctypes.c_uint64()
    ctx = L.Context(0)
    assert raw.gs_poll_status(ctx.handle, None, ctypes.byref(st), ctypes.byref(req)) == L.GS_ERR_INVALID
    assert raw.gs_poll_status(ctx.handle, ctypes.c_void_p(8), ctypes.byref(st), None) == L.GS_ERR_INVALID
    assert b"256-byte aligned" in raw.gs_last_error()
    assert raw.gs_destroy(None) == 0
    ctx.close()


def test_size_limits_and_scheduling_knobs_on_the_host(L):
    raw = L.raw_lib()
    ctx = L.Context(0)
    h = ctx.handle
    # the allocation-free sort refuses more keys than its static scratch holds,
    # and accepts empty or zero-bit sorts without touching a device
    big = ctypes.c_uint64(L.SORT_STATIC_MAX_KEYS + 1)
    p = ctypes.c_void_p(256)
    assert raw.gs_sort_pairs_static(h, p, p, p, p, big, 16, None) == L.GS_ERR_CAPACITY
    assert b"maximum" in raw.gs_last_error()
    assert raw.gs_sort_pairs_static(h, p, p, p, p, ctypes.c_uint64(10), 33, None) == L.GS_ERR_INVALID
    assert raw.gs_sort_pairs_static(h, None, None, None, None, ctypes.c_uint64(0), 16, None) == 0
    assert raw.gs_sort_pairs_static(h, p, p, p, p, ctypes.c_uint64(10), 0, None) == 0
    # scheduling knobs: defaults, accepted values, rejected values leave the setting
    for k, v in (("raster_merge", 0), ("stream_views", 0)):
        assert ctx.get_tuning(k) == v
    ctx.set_tuning("raster_merge", 4096)
    ctx.set_tuning("stream_views", 1)
    assert (ctx.get_tuning("raster_merge"), ctx.get_tuning("stream_views")) == (4096, 1)
    for k, v in (("raster_merge", -1), ("raster_merge", 1 << 32), ("stream_views", 2), ("stream_views", -1)):
        with pytest.raises(L.GsError):
            ctx.set_tuning(k, v)
    assert (ctx.get_tuning("raster_merge"), ctx.get_tuning("stream_views")) == (4096, 1)
    # merging needs workspace for its groups
    cams = (L.GsCamera * 1)()
    cams[0].width, cams[0].height, cams[0].fx, cams[0].fy = 640, 480, 500.0, 500.0
    pc = ctypes.cast(cams, L._PC)
    merged = raw.gs_workspace_bytes(h, pc, 1, 1000, 16, 100000)
    ctx.set_tuning("raster_merge", 0)
    plain = raw.gs_workspace_bytes(h, pc, 1, 1000, 16, 100000)
    assert merged > plain
    ctx.close()
