"""ctypes binding of libxpr.so (include/xpr.h), argument marshalling only.

Every function here has the name of its C entry point and forwards plain
pointers and sizes; all computation happens in the HIP kernels. Loading fails
loudly when the library has not been built: there is no fallback.
"""
from __future__ import annotations

import ctypes
import os

PKG = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(PKG, "libxpr.so")

XPR_OK = 0
XPR_ERR_INVALID_ARG = 1
XPR_ERR_CAPACITY = 2
XPR_ERR_HIP = 3
XPR_ERR_UNSUPPORTED = 4
XPR_SORT_PRESORT = 0
XPR_SORT_FULL = 1
XPR_SORT_BANDS = 2
XPR_SORT_ONESWEEP = 3
XPR_METHOD_3DGS = 0
XPR_METHOD_3DGUT = 1
XPR_METHOD_LINPRIM = 2
XPR_MAX_VIEWS = 32
XPR_MAX_SCENES = 8

_f = ctypes.c_float
_i32 = ctypes.c_int32
_i64 = ctypes.c_int64
_vp = ctypes.c_void_p


class XprCamera(ctypes.Structure):
    _fields_ = [("R", _f * 9), ("t", _f * 3), ("fx", _f), ("fy", _f), ("cx", _f), ("cy", _f),
                ("width", _i32), ("height", _i32)]


class XprConfig(ctypes.Structure):
    _fields_ = [("tile_w", _i32), ("tile_h", _i32), ("lds_batch", _i32), ("sh_degree", _i32),
                ("lowpass", _f), ("alpha_min", _f), ("alpha_max", _f), ("t_min", _f),
                ("z_near", _f), ("fov_clip", _f), ("bg", _f * 3), ("sort_mode", _i32),
                ("no_sync", _i32), ("fwd_ppt", _i32), ("bwd_ppt", _i32),
                ("bwd_lds_batch", _i32), ("persistent", _i32), ("tile_cull", _i32),
                ("opacity_extents", _i32), ("method", _i32), ("bwd_split_walk", _i32)]


class XprScene(ctypes.Structure):
    _fields_ = [("means", _vp), ("scales", _vp), ("quats", _vp), ("opacities", _vp),
                ("sh", _vp), ("n", _i64), ("ld", _i64), ("sh_coeffs", _i32)]


class XprSceneGrad(ctypes.Structure):
    _fields_ = [("means", _vp), ("scales", _vp), ("quats", _vp), ("opacities", _vp),
                ("sh", _vp)]


class XprViews(ctypes.Structure):
    _fields_ = [("scenes", ctypes.POINTER(XprScene)), ("n_scenes", _i32),
                ("cams", ctypes.POINTER(XprCamera)), ("view_scene", ctypes.POINTER(_i32)),
                ("n_views", _i32)]


class XprProjected(ctypes.Structure):
    _fields_ = [("splat", _vp), ("depth", _vp), ("rect", _vp), ("tiles_touched", _vp)]


class XprBins(ctypes.Structure):
    _fields_ = [("keys", _vp), ("vals", _vp), ("tile_ranges", _vp), ("n_isect", _vp),
                ("tile_order", _vp), ("capacity", _i64)]


class XprSizes(ctypes.Structure):
    _fields_ = [("records", _i64), ("tiles", _i64), ("pixels", _i64), ("tile_bits", _i32)]


_LIB = None

# (name, restype, argtypes) of every exported entry point.
_P = ctypes.POINTER
SIGNATURES = {
    "xpr_config_default": (None, [_P(XprConfig)]),
    "xpr_batch_sizes": (_i32, [_P(XprViews), _P(XprConfig), _P(XprSizes)]),
    "xpr_project": (_i32, [_P(XprViews), _P(XprConfig), _P(XprProjected), _vp]),
    "xpr_bin_sort_workspace": (_i32, [_P(XprViews), _P(XprConfig), _i64, _P(ctypes.c_size_t)]),
    "xpr_bin_sort": (_i32, [_P(XprViews), _P(XprConfig), _P(XprProjected), _P(XprBins), _vp,
                            ctypes.c_size_t, _vp]),
    "xpr_render_fwd": (_i32, [_P(XprViews), _P(XprConfig), _P(XprProjected), _P(XprBins), _vp,
                              _vp, _vp, _vp, _vp]),
    "xpr_project_bwd": (_i32, [_P(XprViews), _P(XprConfig), _P(XprProjected), _vp,
                               _P(XprSceneGrad), _i32, _vp]),
    "xpr_render_bwd_workspace": (_i32, [_P(XprViews), _P(XprConfig), _P(ctypes.c_size_t)]),
    "xpr_render_bwd": (_i32, [_P(XprViews), _P(XprConfig), _P(XprProjected), _P(XprBins), _vp,
                              _vp, _vp, _P(XprSceneGrad), _i32, _vp, _vp, ctypes.c_size_t, _vp]),
    "xpr_render_bwd_noalloc": (_i32, [_P(XprViews), _P(XprConfig), _P(XprProjected), _P(XprBins),
                                      _vp, _vp, _vp, _P(XprSceneGrad), _i32, _vp]),
    "xpr_l1_loss": (_i32, [_vp, _vp, _i64, _vp, _vp, _vp]),
    "xpr_last_error": (ctypes.c_char_p, []),
    "xpr_version": (_i32, []),
}


def lib():
    """The loaded library; raises if it was not built (no CPU fallback)."""
    global _LIB
    if _LIB is None:
        if not os.path.exists(LIB_PATH):
            raise ImportError(
                f"{LIB_PATH} is missing: build it with paper_2606_11529_amd.build.build() "
                "(hipcc --offload-arch=gfx950)")
        L = ctypes.CDLL(LIB_PATH)
        for name, (res, args) in SIGNATURES.items():
            fn = getattr(L, name)
            fn.restype = res
            fn.argtypes = args
        _LIB = L
    return _LIB


class XprError(RuntimeError):
    def __init__(self, status: int, fn: str, msg: str):
        super().__init__(f"{fn} failed with status {status}: {msg}")
        self.status = status


def check(status: int, fn: str):
    if status != XPR_OK:
        raise XprError(status, fn, lib().xpr_last_error().decode(errors="replace"))


def xpr_version() -> int:
    return int(lib().xpr_version())


def xpr_config_default() -> XprConfig:
    c = XprConfig()
    lib().xpr_config_default(ctypes.byref(c))
    return c


def xpr_batch_sizes(views, cfg) -> XprSizes:
    s = XprSizes()
    check(lib().xpr_batch_sizes(ctypes.byref(views), ctypes.byref(cfg), ctypes.byref(s)),
          "xpr_batch_sizes")
    return s


def xpr_project(views, cfg, proj, stream) -> None:
    check(lib().xpr_project(ctypes.byref(views), ctypes.byref(cfg), ctypes.byref(proj), stream),
          "xpr_project")


def xpr_bin_sort_workspace(views, cfg, capacity: int) -> int:
    b = ctypes.c_size_t(0)
    check(lib().xpr_bin_sort_workspace(ctypes.byref(views), ctypes.byref(cfg), capacity,
                                       ctypes.byref(b)), "xpr_bin_sort_workspace")
    return int(b.value)


def xpr_bin_sort(views, cfg, proj, bins, ws, ws_bytes, stream) -> int:
    """Returns the raw status (XPR_ERR_CAPACITY is handled by the caller)."""
    st = lib().xpr_bin_sort(ctypes.byref(views), ctypes.byref(cfg), ctypes.byref(proj),
                            ctypes.byref(bins), ws, ws_bytes, stream)
    if st not in (XPR_OK, XPR_ERR_CAPACITY):
        check(st, "xpr_bin_sort")
    return st


def xpr_render_fwd(views, cfg, proj, bins, image, T_final, n_contrib, tile_work, stream) -> None:
    check(lib().xpr_render_fwd(ctypes.byref(views), ctypes.byref(cfg), ctypes.byref(proj),
                               ctypes.byref(bins), image, T_final, n_contrib, tile_work, stream),
          "xpr_render_fwd")


def xpr_project_bwd(views, cfg, proj, grad2d, grads, accumulate, stream) -> None:
    check(lib().xpr_project_bwd(ctypes.byref(views), ctypes.byref(cfg), ctypes.byref(proj),
                                grad2d, grads, accumulate, stream), "xpr_project_bwd")


def xpr_render_bwd_workspace(views, cfg) -> int:
    b = ctypes.c_size_t(0)
    check(lib().xpr_render_bwd_workspace(ctypes.byref(views), ctypes.byref(cfg), ctypes.byref(b)),
          "xpr_render_bwd_workspace")
    return int(b.value)


def xpr_render_bwd(views, cfg, proj, bins, dimage, T_final, n_contrib, grads, accumulate,
                   grad2d, ws, ws_bytes, stream) -> None:
    check(lib().xpr_render_bwd(ctypes.byref(views), ctypes.byref(cfg), ctypes.byref(proj),
                               ctypes.byref(bins), dimage, T_final, n_contrib, grads, accumulate,
                               grad2d, ws, ws_bytes, stream), "xpr_render_bwd")


def xpr_render_bwd_noalloc(views, cfg, proj, bins, dimage, T_final, n_contrib, grads,
                           accumulate, stream) -> None:
    check(lib().xpr_render_bwd_noalloc(ctypes.byref(views), ctypes.byref(cfg),
                                       ctypes.byref(proj), ctypes.byref(bins), dimage, T_final,
                                       n_contrib, grads, accumulate, stream),
          "xpr_render_bwd_noalloc")


def xpr_l1_loss(image, target, n: int, loss, dimage, stream) -> None:
    check(lib().xpr_l1_loss(image, target, n, loss, dimage, stream), "xpr_l1_loss")


def xpr_last_error() -> str:
    return lib().xpr_last_error().decode(errors="replace")
