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
    assert lib.gs_version() == 1
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
