"""The C-ABI library builds for gfx950, loads, and exports every entry point
declared in include/lv.h; argument errors are reported without a GPU."""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


@pytest.fixture(scope="module")
def lvlib():
    import paper_2410_14462_amd as lv
    if not os.path.exists(lv.LIB_PATH):
        from paper_2410_14462_amd import build
        build.build()
    return lv


def declared_functions():
    text = open(os.path.join(ROOT, "include", "lv.h")).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(lv_[a-z_]+)\s*\(", text)))


def test_every_declared_symbol_is_exported(lvlib):
    names = declared_functions()
    assert len(names) >= 15
    L = ctypes.CDLL(lvlib.LIB_PATH)
    for name in names:
        assert hasattr(L, name), name
    assert sorted(lvlib.exported_symbols()) == names


def test_camera_layout_matches_header(lvlib):
    assert ctypes.sizeof(lvlib.lv_camera) == 80
    text = open(os.path.join(ROOT, "include", "lv.h")).read()
    assert "Pinhole camera, 80 bytes" in text


def test_invalid_arguments_fail_without_touching_the_gpu(lvlib):
    L = lvlib.lib()
    out = ctypes.c_void_p()
    assert L.lv_scene_create(None, None, None, None, -1, None, None, ctypes.byref(out)) == 1
    assert b"out of range" in L.lv_last_error()
    assert L.lv_scene_create(None, None, None, None, 10, None, None, ctypes.byref(out)) == 1
    # blending constants other than the compiled ones are refused up front
    opts = lvlib.lv_scene_opts(*lvlib.SCENE_DEFAULTS)
    opts.alpha_min = 0.01
    assert L.lv_scene_create(None, None, None, None, 0, ctypes.byref(opts), None, ctypes.byref(out)) == 4
    assert b"not supported" in L.lv_last_error()
    opts = lvlib.lv_scene_opts(*lvlib.SCENE_DEFAULTS)
    opts.tile = 32
    assert L.lv_scene_create(None, None, None, None, 0, ctypes.byref(opts), None, ctypes.byref(out)) == 4
    # an allocator needs both callbacks
    assert L.lv_set_allocator(lvlib.ALLOC_FN(lambda b, s, c: None), lvlib.FREE_FN(), None) == 1
    assert lvlib.memory_stats() == (0, 0)
    assert L.lv_server_cancel(None, 3) == 1
    assert L.lv_uplift(None, None, 0, None, 0, None, 8, None, None, None) == 1
    assert L.lv_diffuse(None, None, None, 0, 1, 1, None, None) == 1
    assert L.lv_encode(None, 10, 0, 0, None, None, None) == 1
    assert L.lv_version().startswith(b"lv ")
