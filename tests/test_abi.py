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
    assert lib.gsr_render_noalloc(None, None, None) == gsr.GSR_E_INVALID
    assert lib.gsr_trim(None, None) == gsr.GSR_E_INVALID
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


def _c_layout(structs):
    """sizeof and field offsets of header structs as gcc lays them out."""
    import subprocess
    import tempfile
    lines = ['#include <stdio.h>', '#include <stddef.h>', '#include "gsr.h"', "int main(void) {"]
    for cname, fields in structs:
        lines.append(f'printf("{cname} %zu\\n", sizeof({cname}));')
        for f in fields:
            lines.append(f'printf("{cname}.{f} %zu\\n", offsetof({cname}, {f}));')
    lines.append("return 0; }")
    with tempfile.TemporaryDirectory() as d:
        src, exe = os.path.join(d, "l.c"), os.path.join(d, "l")
        with open(src, "w") as f:
            f.write("\n".join(lines))
        subprocess.check_call(["gcc", "-std=c11", "-I", os.path.join(ROOT, "include"), "-o", exe, src])
        out = subprocess.check_output([exe]).decode().split()
    return dict(zip(out[0::2], (int(v) for v in out[1::2])))


def test_struct_layouts_match_header():
    # every ctypes structure of the binding against gcc's layout of include/gsr.h
    pairs = [(gsr.Options, "gsr_options"), (gsr.TuningDesc, "gsr_tuning"), (gsr.SceneDesc, "gsr_scene_desc"),
             (gsr.CameraDesc, "gsr_camera"), (gsr.ObsDesc, "gsr_observation"), (gsr.RenderDesc, "gsr_render_desc"),
             (gsr.BinsOut, "gsr_bins_out"), (gsr.ProjOut, "gsr_proj_out"), (gsr.ServerCfg, "gsr_server_cfg"),
             (gsr.ReqInfo, "gsr_req_info"), (gsr.Stats, "gsr_stats"), (gsr.LidarDesc, "gsr_lidar"),
             (gsr.LidarRenderDesc, "gsr_lidar_desc")]
    lay = _c_layout([(cn, [f for f, _ in py._fields_]) for py, cn in pairs])
    for py, cn in pairs:
        assert C.sizeof(py) == lay[cn], cn
        for f, _ in py._fields_:
            assert getattr(py, f).offset == lay[f"{cn}.{f}"], f"{cn}.{f}"
