"""The C-ABI library loads, exports every entry point of include/xpr.h, and
rejects bad arguments on the host before touching the device (no GPU needed:
none of these calls reaches a HIP launch)."""
import ctypes
import os
import re
import subprocess

import numpy as np
import pytest

from paper_2606_11529_amd import _lib as L

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _declared():
    src = open(os.path.join(ROOT, "include", "xpr.h")).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(xpr_[a-z0-9_]+)\s*\(", src)))


def test_header_and_binding_agree():
    declared = _declared()
    assert len(declared) >= 10
    assert declared == sorted(L.SIGNATURES), (declared, sorted(L.SIGNATURES))


def test_library_exports_every_symbol():
    lib = L.lib()
    for name in _declared():
        assert hasattr(lib, name), name
    assert L.xpr_version() == 1


def test_struct_layouts_match_c_header(tmp_path):
    # sizeof/offsetof of every struct from the C compiler vs the ctypes mirror
    structs = {"xpr_camera": L.XprCamera, "xpr_config": L.XprConfig, "xpr_scene": L.XprScene,
               "xpr_bins": L.XprBins,
               "xpr_scene_grad": L.XprSceneGrad, "xpr_views": L.XprViews,
               "xpr_projected": L.XprProjected, "xpr_sizes": L.XprSizes}
    lines = ['#include <stdio.h>', '#include <stddef.h>', '#include "xpr.h"', "int main(void) {"]
    for cname, py in structs.items():
        lines.append(f'printf("{cname} %zu\\n", sizeof({cname}));')
        for f, _ in py._fields_:
            lines.append(f'printf("{cname}.{f} %zu\\n", offsetof({cname}, {f}));')
    lines.append("return 0; }")
    src = tmp_path / "layout.c"
    src.write_text("\n".join(lines))
    exe = tmp_path / "layout"
    subprocess.run(["gcc", "-D__HIP_PLATFORM_AMD__", "-I", os.path.join(ROOT, "include"),
                    "-I", "/opt/rocm/include", str(src), "-o", str(exe)], check=True)
    out = dict(l.split() for l in subprocess.run([str(exe)], capture_output=True, text=True,
                                                 check=True).stdout.splitlines())
    for cname, py in structs.items():
        assert int(out[cname]) == ctypes.sizeof(py), cname
        for f, _ in py._fields_:
            assert int(out[f"{cname}.{f}"]) == getattr(py, f).offset, (cname, f)


def _views(n=10, W=64, H=48, n_views=1):
    fake = 4096  # never dereferenced by host-only calls
    sc = L.XprScene(fake, fake, fake, fake, fake, n, n, 16)
    cam = L.XprCamera()
    for k, v in enumerate([1, 0, 0, 0, 1, 0, 0, 0, 1]):
        cam.R[k] = v
    cam.fx = cam.fy = 50.0
    cam.cx, cam.cy, cam.width, cam.height = W / 2, H / 2, W, H
    scenes = (L.XprScene * 1)(sc)
    cams = (L.XprCamera * n_views)(*([cam] * n_views))
    vs = (ctypes.c_int32 * n_views)(*([0] * n_views))
    v = L.XprViews(scenes, 1, cams, vs, n_views)
    v._keep = (scenes, cams, vs)
    return v


def test_batch_sizes():
    v = _views(n=10, W=70, H=33, n_views=3)
    c = L.xpr_config_default()
    s = L.xpr_batch_sizes(v, c)
    assert s.records == 30
    assert s.tiles == 3 * 5 * 3
    assert s.pixels == 3 * 70 * 33
    c.tile_w = c.tile_h = 8
    s = L.xpr_batch_sizes(v, c)
    assert s.tiles == 3 * 9 * 5
    c.tile_w = c.tile_h = 32
    s = L.xpr_batch_sizes(v, c)
    assert s.tiles == 3 * 3 * 2
    c.tile_h = 16
    with pytest.raises(L.XprError) as e:
        L.xpr_batch_sizes(v, c)
    assert e.value.status == L.XPR_ERR_INVALID_ARG


@pytest.mark.parametrize("field,value", [
    ("tile_w", 12), ("lds_batch", 100), ("sh_degree", 4), ("alpha_min", 0.0),
    ("alpha_max", 1.5), ("t_min", 0.0), ("z_near", 0.0), ("sort_mode", 7), ("lowpass", -1.0),
    ("fwd_ppt", 3), ("bwd_ppt", 8), ("bwd_lds_batch", 100)])
def test_invalid_config_rejected(field, value):
    v = _views()
    c = L.xpr_config_default()
    setattr(c, field, value)
    with pytest.raises(L.XprError) as e:
        L.xpr_project(v, c, L.XprProjected(4096, 4096, 4096, 4096), None)
    assert e.value.status == L.XPR_ERR_INVALID_ARG
    assert L.xpr_last_error()


def test_invalid_views_rejected():
    c = L.xpr_config_default()
    v = _views(n_views=1)
    v.n_views = 0
    with pytest.raises(L.XprError):
        L.xpr_batch_sizes(v, c)
    v = _views()
    v._keep[1][0].width = 0
    with pytest.raises(L.XprError):
        L.xpr_batch_sizes(v, c)
    v = _views()
    v._keep[2][0] = 3   # scene index out of range
    with pytest.raises(L.XprError):
        L.xpr_batch_sizes(v, c)
    v = _views()
    v._keep[0][0].sh_coeffs = 4  # degree 3 needs 16
    with pytest.raises(L.XprError):
        L.xpr_batch_sizes(v, c)


def test_misaligned_projected_rejected():
    v = _views()
    c = L.xpr_config_default()
    with pytest.raises(L.XprError) as e:
        L.xpr_project(v, c, L.XprProjected(4100, 4096, 4096, 4096), None)
    assert "misaligned" in str(e.value)


def test_workspace_queries_host_only():
    v = _views(n=1000)
    c = L.xpr_config_default()
    a = L.xpr_bin_sort_workspace(v, c, 100_000)
    b = L.xpr_bin_sort_workspace(v, c, 200_000)
    assert 0 < a < b
    c.sort_mode = L.XPR_SORT_FULL
    assert L.xpr_bin_sort_workspace(v, c, 100_000) > 0
    # the split backward's tile data (128 words + 1 per tile, in 256-byte
    # units), then 36 bytes per record
    meta = -(-(128 + 12) * 4 // 256) * 256
    assert L.xpr_render_bwd_workspace(v, c) == meta + 9 * 4 * 1000
    # 3DGUT and LinPrim: 16 floats per record
    c.method = L.XPR_METHOD_3DGUT
    assert L.xpr_render_bwd_workspace(v, c) == meta + 16 * 4 * 1000
    c.method = L.XPR_METHOD_LINPRIM
    assert L.xpr_render_bwd_workspace(v, c) == meta + 16 * 4 * 1000
    c.method = L.XPR_METHOD_3DGS
    with pytest.raises(L.XprError):
        L.xpr_bin_sort_workspace(v, c, -1)


def test_bin_sort_rejects_small_workspace():
    v = _views(n=100)
    c = L.xpr_config_default()
    bins = L.XprBins(None, 4096, 4096, 4096, None, 1000)
    st = L.lib().xpr_bin_sort(ctypes.byref(v), ctypes.byref(c),
                              ctypes.byref(L.XprProjected(4096, 4096, 4096, 4096)),
                              ctypes.byref(bins), 4096, 16, None)
    assert st == L.XPR_ERR_INVALID_ARG
    assert "workspace" in L.xpr_last_error()


def test_noalloc_backward_rejects_more_records_than_its_scratch():
    # 1,835,008 records fit the 63 MiB of the static scratch left after the
    # split backward's tile data (36 bytes each); a second view of a 1M
    # scene is refused on the host, before any device call
    c = L.xpr_config_default()
    grads = (L.XprSceneGrad * 1)(L.XprSceneGrad(4096, 4096, 4096, 4096, 4096))
    args = (L.XprProjected(4096, 4096, 4096, 4096), L.XprBins(None, 4096, 4096, 4096, None, 10))
    v = _views(n=1_000_000, n_views=2)
    st = L.lib().xpr_render_bwd_noalloc(ctypes.byref(v), ctypes.byref(c), ctypes.byref(args[0]),
                                        ctypes.byref(args[1]), 4096, 4096, 4096, grads, 0, None)
    assert st == L.XPR_ERR_CAPACITY
    msg = L.xpr_last_error()
    assert "2000000 records" in msg and "1835008 records" in msg
    st = L.lib().xpr_render_bwd_noalloc(ctypes.byref(v), ctypes.byref(c), ctypes.byref(args[0]),
                                        ctypes.byref(args[1]), 4096, 4096, 4096, None, 0, None)
    assert st == L.XPR_ERR_INVALID_ARG and "grads" in L.xpr_last_error()
    # 3DGUT's 64 bytes per record: 1,032,192 fit, one view of 1.1M does not
    c.method = L.XPR_METHOD_3DGUT
    v = _views(n=1_100_000, n_views=1)
    st = L.lib().xpr_render_bwd_noalloc(ctypes.byref(v), ctypes.byref(c), ctypes.byref(args[0]),
                                        ctypes.byref(args[1]), 4096, 4096, 4096, grads, 0, None)
    assert st == L.XPR_ERR_CAPACITY
    msg = L.xpr_last_error()
    assert "1100000 records" in msg and "1032192 records" in msg
