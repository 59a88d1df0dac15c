"""Device-side Python API over the C-ABI: scenes, batches of views and the
four stages (project, bin_sort, render_fwd, render_bwd).

PyTorch provides device memory and the stream; every stage runs in the HIP
kernels of libxpr.so. Buffers are SoA float32 tensors laid out as the C-ABI
expects (component-major, leading dimension ld).
"""
from __future__ import annotations

import ctypes
import dataclasses
from typing import List, Optional, Sequence

import numpy as np
import torch

from . import _lib as L


@dataclasses.dataclass
class Config:
    """Method constants and tuning knobs (xpr_config)."""
    tile: int = 16
    lds_batch: int = 256
    sh_degree: int = 3
    lowpass: float = 0.3
    alpha_min: float = 1.0 / 255.0
    alpha_max: float = 0.99
    t_min: float = 1e-4
    z_near: float = 0.2
    fov_clip: float = 1.3
    bg: tuple = (0.0, 0.0, 0.0)
    sort_mode: str = "presort"  # "presort", "full", "bands" or "onesweep"
    no_sync: bool = False
    fwd_ppt: int = 2            # pixels per thread, forward (16x16 tiles)
    bwd_ppt: int = 4            # pixels per thread, backward (16x16 tiles)
    bwd_lds_batch: int = 0      # LDS batch of the backward (0: lds_batch)
    persistent: bool = False    # persistent render grids over the tile order
    tile_order: bool = False    # launch tiles longest list first (implied by persistent)
    tile_cull: bool = False     # per-(Gaussian, tile) cull of XPR-3DGS in the binning
    opacity_extents: bool = False  # rect from the alpha >= alpha_min ellipse, not 3 sigma
    method: str = "3dgs"        # "3dgs", "3dgut" or "linprim"
    bwd_split_walk: int = 2048  # backward: tiles whose walk reaches this go as four bands

    def to_c(self) -> L.XprConfig:
        c = L.XprConfig()
        c.tile_w = c.tile_h = int(self.tile)
        c.lds_batch = int(self.lds_batch)
        c.sh_degree = int(self.sh_degree)
        c.lowpass = self.lowpass
        c.alpha_min = self.alpha_min
        c.alpha_max = self.alpha_max
        c.t_min = self.t_min
        c.z_near = self.z_near
        c.fov_clip = self.fov_clip
        for k in range(3):
            c.bg[k] = float(self.bg[k])
        modes = {"presort": L.XPR_SORT_PRESORT, "full": L.XPR_SORT_FULL, "bands": L.XPR_SORT_BANDS,
                 "onesweep": L.XPR_SORT_ONESWEEP}
        if self.sort_mode not in modes:
            raise ValueError(f"unknown sort_mode {self.sort_mode!r}")
        c.sort_mode = modes[self.sort_mode]
        c.no_sync = 1 if self.no_sync else 0
        c.fwd_ppt = int(self.fwd_ppt)
        c.bwd_ppt = int(self.bwd_ppt)
        c.bwd_lds_batch = int(self.bwd_lds_batch)
        c.persistent = 1 if self.persistent else 0
        c.tile_cull = 1 if self.tile_cull else 0
        c.opacity_extents = 1 if self.opacity_extents else 0
        methods = {"3dgs": L.XPR_METHOD_3DGS, "3dgut": L.XPR_METHOD_3DGUT,
                   "linprim": L.XPR_METHOD_LINPRIM}
        if self.method not in methods:
            raise ValueError(f"unknown method {self.method!r}")
        c.method = methods[self.method]
        c.bwd_split_walk = int(self.bwd_split_walk)
        return c


def _ptr(t: Optional[torch.Tensor]):
    return None if t is None else ctypes.c_void_p(t.data_ptr())


def _stream() -> ctypes.c_void_p:
    return ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)


class Scene:
    """Gaussians resident on the device (SoA float32)."""

    def __init__(self, means, scales, quats, opacities, sh):
        self.n = int(opacities.shape[-1])
        shapes = ((means, (3, self.n)), (scales, (3, self.n)), (quats, (4, self.n)),
                  (opacities, (self.n,)))
        for t, shp in shapes:
            if tuple(t.shape) != shp or t.dtype != torch.float32:
                raise ValueError(f"expected float32 {shp}, got {t.dtype} {tuple(t.shape)}")
        if sh.dim() != 3 or sh.shape[1] != 3 or sh.shape[2] != self.n or sh.dtype != torch.float32:
            raise ValueError(f"sh must be float32 [K, 3, {self.n}]")
        self.means, self.scales, self.quats = (t.contiguous() for t in (means, scales, quats))
        self.opacities, self.sh = opacities.contiguous(), sh.contiguous()
        self.ld = self.n

    @classmethod
    def from_host(cls, scene, device="cuda") -> "Scene":
        """From a synth.Scene (numpy SoA arrays)."""
        t = lambda a: torch.from_numpy(np.ascontiguousarray(a)).to(device)
        return cls(t(scene.means), t(scene.scales), t(scene.quats), t(scene.opacities),
                   t(scene.sh))

    @property
    def sh_coeffs(self) -> int:
        return int(self.sh.shape[0])

    def to_c(self) -> L.XprScene:
        s = L.XprScene()
        s.means, s.scales, s.quats = (t.data_ptr() for t in (self.means, self.scales, self.quats))
        s.opacities, s.sh = self.opacities.data_ptr(), self.sh.data_ptr()
        s.n, s.ld, s.sh_coeffs = self.n, self.ld, self.sh_coeffs
        return s

    def zeros_like_grads(self):
        return dict(means=torch.zeros_like(self.means), scales=torch.zeros_like(self.scales),
                    quats=torch.zeros_like(self.quats),
                    opacities=torch.zeros_like(self.opacities), sh=torch.zeros_like(self.sh))

    def nbytes(self) -> int:
        return sum(t.numel() * 4 for t in (self.means, self.scales, self.quats, self.opacities,
                                            self.sh))


def camera_to_c(cam) -> L.XprCamera:
    c = L.XprCamera()
    R = np.asarray(cam.R, dtype=np.float64).reshape(9)
    t = np.asarray(cam.t, dtype=np.float64).reshape(3)
    for k in range(9):
        c.R[k] = float(R[k])
    for k in range(3):
        c.t[k] = float(t[k])
    c.fx, c.fy, c.cx, c.cy = float(cam.fx), float(cam.fy), float(cam.cx), float(cam.cy)
    c.width, c.height = int(cam.width), int(cam.height)
    return c


class Views:
    """A batch: n_views cameras over n_scenes scenes, with the offsets of
    every view in the concatenated record, tile and pixel buffers."""

    def __init__(self, scenes: Sequence[Scene], cams: Sequence, view_scene: Sequence[int],
                 cfg: Config):
        assert 1 <= len(cams) <= L.XPR_MAX_VIEWS and 1 <= len(scenes) <= L.XPR_MAX_SCENES
        self.scenes = list(scenes)
        self.cams = list(cams)
        self.view_scene = [int(s) for s in view_scene]
        self._scenes_c = (L.XprScene * len(scenes))(*[s.to_c() for s in scenes])
        self._cams_c = (L.XprCamera * len(cams))(*[camera_to_c(c) for c in cams])
        self._vs_c = (ctypes.c_int32 * len(cams))(*self.view_scene)
        self.c = L.XprViews(self._scenes_c, len(scenes), self._cams_c, self._vs_c, len(cams))
        self.cfg_c = cfg.to_c()
        sz = L.xpr_batch_sizes(self.c, self.cfg_c)
        self.records, self.tiles, self.pixels = int(sz.records), int(sz.tiles), int(sz.pixels)
        self.tile_bits = int(sz.tile_bits)
        self.rec_off, self.tile_off, self.pix_off = [], [], []
        r = t = p = 0
        for v, cam in enumerate(cams):
            self.rec_off.append(r)
            self.tile_off.append(t)
            self.pix_off.append(p)
            r += self.scenes[self.view_scene[v]].n
            t += (-(-cam.width // cfg.tile)) * (-(-cam.height // cfg.tile))
            p += cam.width * cam.height
        assert (r, t, p) == (self.records, self.tiles, self.pixels)

    @property
    def n_views(self) -> int:
        return len(self.cams)

    def image(self, flat: torch.Tensor, v: int) -> torch.Tensor:
        cam = self.cams[v]
        o = 3 * self.pix_off[v]
        return flat[o:o + 3 * cam.width * cam.height].view(3, cam.height, cam.width)

    def plane(self, flat: torch.Tensor, v: int) -> torch.Tensor:
        cam = self.cams[v]
        o = self.pix_off[v]
        return flat[o:o + cam.width * cam.height].view(cam.height, cam.width)


@dataclasses.dataclass
class Projected:
    splat: torch.Tensor   # [R, 12] f32 (3DGS), [R, 24] (3DGUT) or [R, 20] (LinPrim)
    depth: torch.Tensor   # [R] f32
    rect: torch.Tensor    # [R, 4] i16
    tc: torch.Tensor      # [R] i32

    def to_c(self) -> L.XprProjected:
        return L.XprProjected(self.splat.data_ptr(), self.depth.data_ptr(), self.rect.data_ptr(),
                              self.tc.data_ptr())


@dataclasses.dataclass
class Bins:
    vals: torch.Tensor     # [cap] i32
    ranges: torch.Tensor   # [tiles, 2] i32
    n_isect: torch.Tensor  # [1] i64 (device)
    keys: Optional[torch.Tensor] = None  # [cap] i64 (bits of uint64)
    capacity: int = 0
    count_cache: int = -1  # host copy of n_isect once read (-1: not read yet)
    tile_order: Optional[torch.Tensor] = None  # [tiles + 1] i32

    @property
    def count(self) -> int:
        """Host copy of n_isect, read (one stream sync) the first time it is
        asked for after a binning, so a frame that never asks does not wait."""
        if self.count_cache < 0:
            self.count_cache = int(self.n_isect.item())
        return self.count_cache

    def to_c(self) -> L.XprBins:
        return L.XprBins(self.keys.data_ptr() if self.keys is not None else None,
                         self.vals.data_ptr(), self.ranges.data_ptr(), self.n_isect.data_ptr(),
                         self.tile_order.data_ptr() if self.tile_order is not None else None,
                         self.capacity)


@dataclasses.dataclass
class Frame:
    image: torch.Tensor    # [3 * pixels] f32 (view-planar)
    T_final: torch.Tensor  # [pixels] f32
    n_contrib: torch.Tensor  # [pixels] i32


def splat_floats(cfg: "Config") -> int:
    """Floats per projected record: 12 for 3DGS, 24 for 3DGUT, 20 for LinPrim."""
    return {"3dgut": 24, "linprim": 20}.get(cfg.method, 12)


def grad2d_floats(cfg: "Config") -> int:
    """Floats per record of the backward's shader-data gradient: 9 for 3DGS
    (mean2D, conic, opacity, colour), 16 for 3DGUT (o', colour, ro, M) and
    LinPrim (mean2D, sigma, colour, the rows of A^-1, one zero)."""
    return 9 if cfg.method == "3dgs" else 16


def empty_projected(n: int, device, floats: int = 12) -> Projected:
    n1 = max(n, 1)
    return Projected(torch.empty((n1, floats), dtype=torch.float32, device=device),
                     torch.empty(n1, dtype=torch.float32, device=device),
                     torch.empty((n1, 4), dtype=torch.int16, device=device),
                     torch.empty(n1, dtype=torch.int32, device=device))


def xpr_project(views: Views, cfg: Config, out: Optional[Projected] = None) -> Projected:
    dev = views.scenes[0].means.device
    nf = splat_floats(cfg)
    if out is not None and (out.splat.shape[1] != nf or out.splat.shape[0] < views.records):
        raise ValueError(f"out.splat must be [>= {views.records}, {nf}] for method {cfg.method}")
    out = out or empty_projected(views.records, dev, nf)
    L.xpr_project(views.c, views.cfg_c, out.to_c(), _stream())
    return out


class Workspace:
    """Growing device scratch reused across calls (caller-owned memory)."""

    def __init__(self):
        self.buf = {}

    def get(self, name: str, nbytes: int, device) -> torch.Tensor:
        b = self.buf.get(name)
        if b is None or b.numel() < nbytes:
            b = torch.empty(max(nbytes, 256), dtype=torch.uint8, device=device)
            self.buf[name] = b
        return b


_WS = Workspace()


def xpr_bin_sort(views: Views, cfg: Config, proj: Projected, capacity: Optional[int] = None,
                 want_keys: bool = False, ws: Optional[Workspace] = None,
                 out: Optional[Bins] = None, want_order: Optional[bool] = None) -> Bins:
    """Binning with a host-side capacity retry on XPR_ERR_CAPACITY. The
    longest-first tile order is produced when ``want_order`` (default: when
    the config asks for it or is persistent)."""
    ws = ws or _WS
    dev = proj.splat.device
    want_order = (cfg.persistent or cfg.tile_order) if want_order is None else want_order
    cap = capacity if capacity is not None else max(1024, 16 * views.records)
    if out is not None and out.capacity >= cap:
        cap = out.capacity
    while True:
        if (out is None or out.capacity < cap or (want_keys and out.keys is None)
                or out.ranges.shape[0] < views.tiles
                or (want_order and (out.tile_order is None
                                    or out.tile_order.numel() < views.tiles + 1))):
            out = Bins(vals=torch.empty(max(cap, 1), dtype=torch.int32, device=dev),
                       ranges=torch.empty((max(views.tiles, 1), 2), dtype=torch.int32, device=dev),
                       n_isect=torch.zeros(1, dtype=torch.int64, device=dev),
                       keys=torch.empty(max(cap, 1), dtype=torch.int64, device=dev) if want_keys else None,
                       capacity=cap,
                       tile_order=torch.empty(views.tiles + 1, dtype=torch.int32, device=dev)
                       if want_order else None)
        bc = out.to_c()
        if not want_keys:
            bc.keys = None
        if not want_order:
            bc.tile_order = None
        nbytes = L.xpr_bin_sort_workspace(views.c, views.cfg_c, cap)
        wsb = ws.get("bin", nbytes, dev)
        st = L.xpr_bin_sort(views.c, views.cfg_c, proj.to_c(), bc, _ptr(wsb), wsb.numel(),
                            _stream())
        if st == L.XPR_OK:
            out.count_cache = -1
            return out
        need = int(out.n_isect.item())
        cap = int(need * 1.125) + 1024
        out = None


def xpr_render_fwd(views: Views, cfg: Config, proj: Projected, bins: Bins,
                   out: Optional[Frame] = None, tile_work: Optional[torch.Tensor] = None) -> Frame:
    dev = proj.splat.device
    if out is None:
        out = Frame(torch.empty(3 * views.pixels, dtype=torch.float32, device=dev),
                    torch.empty(views.pixels, dtype=torch.float32, device=dev),
                    torch.empty(views.pixels, dtype=torch.int32, device=dev))
    L.xpr_render_fwd(views.c, views.cfg_c, proj.to_c(), bins.to_c(), _ptr(out.image),
                     _ptr(out.T_final), _ptr(out.n_contrib), _ptr(tile_work), _stream())
    return out


def _grads_c(grads):
    return (L.XprSceneGrad * len(grads))(*[
        L.XprSceneGrad(g["means"].data_ptr(), g["scales"].data_ptr(), g["quats"].data_ptr(),
                       g["opacities"].data_ptr(), g["sh"].data_ptr()) for g in grads])


def xpr_render_bwd(views: Views, cfg: Config, proj: Projected, bins: Bins, frame: Frame,
                   dimage: torch.Tensor, grads: Optional[List[dict]] = None,
                   accumulate: bool = False, want_grad2d: bool = False,
                   ws: Optional[Workspace] = None, params: bool = True,
                   grad2d: Optional[torch.Tensor] = None):
    """Returns (grads per scene or None, grad2d or None). With params=False
    only the compositing backward runs and grad2d [records, grad2d_floats]
    is returned."""
    ws = ws or _WS
    dev = proj.splat.device
    if params and grads is None:
        grads = [s.zeros_like_grads() for s in views.scenes]
    arr = _grads_c(grads) if params else None
    dimage = dimage.contiguous()
    if grad2d is None and (want_grad2d or not params):
        grad2d = torch.empty((max(views.records, 1), grad2d_floats(cfg)), dtype=torch.float32,
                             device=dev)
    nbytes = L.xpr_render_bwd_workspace(views.c, views.cfg_c)
    wsb = ws.get("bwd", nbytes, dev)
    L.xpr_render_bwd(views.c, views.cfg_c, proj.to_c(), bins.to_c(), _ptr(dimage),
                     _ptr(frame.T_final), _ptr(frame.n_contrib), arr, 1 if accumulate else 0,
                     _ptr(grad2d), _ptr(wsb), wsb.numel(), _stream())
    return (grads if params else None), grad2d


def xpr_render_bwd_noalloc(views: Views, cfg: Config, proj: Projected, bins: Bins, frame: Frame,
                           dimage: torch.Tensor, grads: List[dict], accumulate: bool = False):
    """The backward into caller-owned parameter gradients with the library's
    static device scratch for the 2D gradients: nothing is allocated (the
    caller passes every buffer)."""
    L.xpr_render_bwd_noalloc(views.c, views.cfg_c, proj.to_c(), bins.to_c(), _ptr(dimage),
                             _ptr(frame.T_final), _ptr(frame.n_contrib), _grads_c(grads),
                             1 if accumulate else 0, _stream())
    return grads


def xpr_project_bwd(views: Views, cfg: Config, proj: Projected, grad2d: torch.Tensor,
                    grads: Optional[List[dict]] = None, accumulate: bool = False):
    if grads is None:
        grads = [s.zeros_like_grads() for s in views.scenes]
    L.xpr_project_bwd(views.c, views.cfg_c, proj.to_c(), _ptr(grad2d), _grads_c(grads),
                      1 if accumulate else 0, _stream())
    return grads


def xpr_l1_loss(image: torch.Tensor, target: torch.Tensor,
                loss: Optional[torch.Tensor] = None,
                dimage: Optional[torch.Tensor] = None):
    """L1 loss mean |image - target| (one device float) and its gradient
    sign(image - target) / n, in one kernel pass; image and target are
    contiguous float32 tensors of the same size."""
    if image.dtype != torch.float32 or target.dtype != torch.float32:
        raise TypeError("image and target must be float32")
    if not (image.is_contiguous() and target.is_contiguous()) or image.numel() != target.numel():
        raise ValueError("image and target must be contiguous and of equal size")
    n = image.numel()
    if loss is None:
        loss = torch.empty(1, dtype=torch.float32, device=image.device)
    if dimage is None:
        dimage = torch.empty_like(image)
    L.xpr_l1_loss(_ptr(image), _ptr(target), n, _ptr(loss), _ptr(dimage), _stream())
    return loss, dimage


def render(scene: Scene, cam, cfg: Config, want_keys: bool = False):
    """One view: returns (image [3,H,W], state dict)."""
    views = Views([scene], [cam], [0], cfg)
    proj = xpr_project(views, cfg)
    bins = xpr_bin_sort(views, cfg, proj, want_keys=want_keys)
    frame = xpr_render_fwd(views, cfg, proj, bins)
    return views.image(frame.image, 0), dict(views=views, proj=proj, bins=bins, frame=frame)


def render_batch(scene, cams, cfg: Config, view_scene=None):
    """Many views, one launch per stage: ``scene`` is a Scene or a list of
    them and view v renders scene ``view_scene[v]`` (default 0), cameras of
    any sizes. Returns ([image [3,H,W] per view], state dict)."""
    scenes = list(scene) if isinstance(scene, (list, tuple)) else [scene]
    cams = list(cams)
    vs = [0] * len(cams) if view_scene is None else [int(i) for i in view_scene]
    views = Views(scenes, cams, vs, cfg)
    proj = xpr_project(views, cfg)
    bins = xpr_bin_sort(views, cfg, proj)
    frame = xpr_render_fwd(views, cfg, proj, bins)
    images = [views.image(frame.image, v) for v in range(len(cams))]
    return images, dict(views=views, proj=proj, bins=bins, frame=frame)
