"""CPU checks of the C ABI: the library loads, exports every entry point the
public header declares, and rejects bad arguments before any device work.
No compute call is made here."""
import ctypes as C
import os
import re

import numpy as np
import pytest

from paper_2604_25459_amd import gsr

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def declared_functions():
    names = set()
    for fn in os.listdir(os.path.join(ROOT, "include")):
        if fn.endswith(".h"):
            txt = open(os.path.join(ROOT, "include", fn)).read()
            txt = re.sub(r"/\*.*?\*/", "", txt, flags=re.S)
            names |= set(re.findall(r"\b(gsr_[a-z_]+)\s*\(", txt))
    return sorted(names)


def test_library_exports_every_declared_symbol():
    lib = gsr.load()
    names = declared_functions()
    assert "gsr_render" in names and "gsr_create" in names
    for name in names:
        assert hasattr(lib, name), name
    # the binding knows every declared function with an explicit signature
    assert set(names) <= set(gsr.SIGNATURES), set(names) - set(gsr.SIGNATURES)


def test_version_and_error_strings():
    lib = gsr.load()
    assert b"gfx950" in lib.gsr_version()
    assert lib.gsr_render(None, None, None) == gsr.GSR_E_INVALID
    assert b"ctx" in lib.gsr_last_error()


def test_null_arguments_rejected():
    lib = gsr.load()
    assert lib.gsr_create(0, None, None) == gsr.GSR_E_INVALID
    assert lib.gsr_scene_create(None, None, None) == gsr.GSR_E_INVALID
    assert lib.gsr_scene_destroy(None, 1) == gsr.GSR_E_INVALID
    assert lib.gsr_render_plain(None, None, None) == gsr.GSR_E_INVALID
    assert lib.gsr_debug_bins(None, None, 0, None) == gsr.GSR_E_INVALID
    assert lib.gsr_debug_project(None, None, 0, None) == gsr.GSR_E_INVALID
    assert lib.gsr_scene_info(None, 1, None, None, None) == gsr.GSR_E_INVALID
    assert lib.gsr_stage_times(None, None, 0, 0) == gsr.GSR_E_INVALID
    assert lib.gsr_server_create(None, None, None) == gsr.GSR_E_INVALID
    assert lib.gsr_submit(None, None, None) == gsr.GSR_E_INVALID
    assert lib.gsr_wait(None, 1, 0, None) == gsr.GSR_E_INVALID
    assert lib.gsr_server_stats(None, None) == gsr.GSR_E_INVALID
    assert lib.gsr_server_destroy(None) == gsr.GSR_OK
    assert lib.gsr_autotune(None, None, None, None) == gsr.GSR_E_INVALID
    assert lib.gsr_tuning_get(None, None, None) == gsr.GSR_E_INVALID
    assert lib.gsr_tuning_set(None, None, None) == gsr.GSR_E_INVALID
    assert lib.gsr_tuning_save(None, None) == gsr.GSR_E_INVALID
    assert lib.gsr_tuning_load(None, None) == gsr.GSR_E_INVALID
    assert lib.gsr_destroy(None) == gsr.GSR_OK


def test_bad_options_rejected_before_device():
    lib = gsr.load()
    h = C.c_void_p()
    for opt in (gsr.Options(tile_size=12), gsr.Options(images_per_thread=99), gsr.Options(cutoff=0.5),
                gsr.Options(chunk_bytes=1024)):
        assert lib.gsr_create(0, C.byref(opt), C.byref(h)) == gsr.GSR_E_INVALID
        assert h.value is None


def test_create_without_gpu_reports_device_error():
    import torch
    if torch.cuda.is_available():
        pytest.skip("a GPU is present")
    lib = gsr.load()
    h = C.c_void_p()
    assert lib.gsr_create(0, None, C.byref(h)) == gsr.GSR_E_DEVICE


def test_struct_layouts_match_header():
    # sizes computed from the C declarations (LP64): a mismatch would corrupt every call
    assert C.sizeof(gsr.Options) == 4 + 4 + 8 + 4 + 4 + 4 + 24 + 4
    assert C.sizeof(gsr.TuningDesc) == 6 * 4 + 16
    assert C.sizeof(gsr.SceneDesc) == 8 + 4 * 4 + 8 * 6
    assert C.sizeof(gsr.CameraDesc) == 7 * 4
    assert C.sizeof(gsr.RenderDesc) == 8 + 4 + 4 + 8 * 3 + 12 + 4 + 8 * 4
    assert C.sizeof(gsr.BinsOut) == 8 * 5 + 8 + 8 + 4 + 4 + 8
    assert C.sizeof(gsr.ProjOut) == 8 * 4
    assert C.sizeof(gsr.ServerCfg) == 4 + 4 + 8 + 32
    assert C.sizeof(gsr.ReqInfo) == 4 + 4 + 8 + 4 + 4 + 8 * 4
    assert C.sizeof(gsr.Stats) == 8 * 8 + 8 * 5
