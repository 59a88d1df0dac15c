"""FP64 CPU oracle for 3DGS tile splatting, forward and backward.

TEST INFRASTRUCTURE ONLY: the tests, the smoke check and the bench's
CPU-baseline leg may use it; the product path never imports it.

Two independent forms of the same definition:
  * ``liboracle.so`` (oracle.cpp): the tiled pipeline in double precision,
    project -> bin (prefix sum, replicate, sort, ranges) -> composite, and the
    analytic backward of every stage;
  * ``brute``: per-pixel brute force (numpy / torch float64) with no pairs,
    no sort and no ranges, differentiable with torch autograd.

Citations are to the paper (XPR, arxiv 2606.11529): Background section
(blending), Listing "Implementation of XPR-3DGS" (project/evaluate/
tile_cull), section "Rasterizer" (replicate, tile id, sort, bounds),
Algorithm 1 (shader loop).
"""
from __future__ import annotations

import ctypes
import dataclasses
import os

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
_LIB = None


@dataclasses.dataclass
class OracleConfig:
    """Constants of the method (readings listed in the design notes)."""
    tile_w: int = 16
    tile_h: int = 16
    sh_degree: int = 3
    lowpass: float = 0.3            # added to both diagonal entries of cov2D
    alpha_min: float = 1.0 / 255.0  # alpha_thresh of the listing
    alpha_max: float = 0.99
    t_min: float = 1e-4             # stop before blending if T(1-a) < t_min
    z_near: float = 0.2
    fov_clip: float = 1.3           # Jacobian clamp at fov_clip*tan(fov/2)
    bg: tuple = (0.0, 0.0, 0.0)
    tile_cull: bool = False         # per-(Gaussian, tile) cull of XPR-3DGS
    opacity_extents: bool = False   # rect from the alpha >= alpha_min ellipse (not 3 sigma)
    method: str = "3dgs"            # "3dgs" (EWA), "3dgut" (unscented transform, ray evaluate)
    #                                 or "linprim" (octahedra, slab chords, Beer-Lambert)

    def proj_cfg(self):
        return np.array([self.lowpass, self.alpha_min, self.z_near, self.fov_clip,
                         1.0 if self.opacity_extents else 0.0], dtype=np.float64)

    def gut_cfg(self):
        return np.array([self.lowpass, self.alpha_min, self.z_near,
                         1.0 if self.opacity_extents else 0.0], dtype=np.float64)

    def render_cfg(self):
        return np.array([self.alpha_min, self.alpha_max, self.t_min, *self.bg],
                        dtype=np.float64)


def lib():
    global _LIB
    if _LIB is None:
        path = os.path.join(HERE, "liboracle.so")
        if not os.path.exists(path):
            from . import build as _b
            _b.build()
        L = ctypes.CDLL(path)
        P = ctypes.c_void_p
        i64, i32 = ctypes.c_int64, ctypes.c_int
        L.orc_project.argtypes = [i64, P, P, P, P, P, i32, P, i32, i32, P, i32, i32, i32,
                                  P, P, P, P, P, P, P]
        L.orc_project.restype = None
        L.orc_bin.argtypes = [i64, P, P, P, i32, i32, i64, P, P, P, P, P, i32, i32, i32, i32,
                              i32, i32, ctypes.c_double, P, P, P]
        L.orc_bin.restype = i64
        L.orc_tile_cull.argtypes = [i64, P, i32, P, i32, i32, i32, i32, ctypes.c_double, i32, P,
                                    P, P, P]
        L.orc_tile_cull.restype = None
        L.orc_render_fwd.argtypes = [i32, i32, i32, i32, P, P, P, P, P, P, P, P, P, P, P, P]
        L.orc_render_fwd.restype = None
        L.orc_render_bwd.argtypes = [i32, i32, i32, i32, i64, P, P, P, P, P, P]
        L.orc_render_bwd.restype = None
        L.orc_project_bwd.argtypes = [i64, P, P, P, P, P, i32, P, i32, i32, P, i32, i32, i32,
                                      P, P, P, P, P, P]
        L.orc_project_bwd.restype = None
        L.orc_project_gut.argtypes = [i64, P, P, P, P, P, P, i32, i32, P, i32, i32, i32,
                                      P, P, P, P, P, P]
        L.orc_project_gut.restype = None
        L.orc_render_fwd_gut.argtypes = [i32, i32, i32, i32, P, P, P, P, P, P, P, P, P, P, P]
        L.orc_render_fwd_gut.restype = None
        L.orc_gut_response.argtypes = [i64, P, P, P, i32, i32, P]
        L.orc_gut_response.restype = None
        L.orc_project_lin.argtypes = [i64, P, P, P, P, P, P, i32, i32, P, i32, i32, i32,
                                      P, P, P, P, P]
        L.orc_project_lin.restype = None
        L.orc_lin_chord.argtypes = [i64, P, P, P]
        L.orc_lin_chord.restype = None
        L.orc_render_fwd_lin.argtypes = [i32, i32, i32, i32, P, P, P, P, P, P, P, P, P, P]
        L.orc_render_fwd_lin.restype = None
        L.orc_render_bwd_lin.argtypes = [i32, i32, i32, i32, i64, P, P, P, P, P, P]
        L.orc_render_bwd_lin.restype = None
        L.orc_project_bwd_lin.argtypes = [i64, P, P, P, P, P, i32, P, i32, i32, P, i32, i32,
                                          i32, P, P, P, P, P, P]
        L.orc_project_bwd_lin.restype = None
        L.orc_render_bwd_gut.argtypes = [i32, i32, i32, i32, i64, P, P, P, P, P, P, P]
        L.orc_render_bwd_gut.restype = None
        L.orc_project_bwd_gut.argtypes = [i64, P, P, P, P, P, i32, P, i32, i32, P, i32, i32, i32,
                                          P, P, P, P, P, P]
        L.orc_project_bwd_gut.restype = None
        L.orc_sh_basis.argtypes = [i32, P, P, P]
        L.orc_sh_basis.restype = None
        L.orc_num_threads.restype = i32
        L.orc_set_num_threads.argtypes = [i32]
        L.orc_set_num_threads.restype = None
        _LIB = L
    return _LIB


def _p(a):
    return None if a is None else a.ctypes.data_as(ctypes.c_void_p)


def _f64(a):
    return np.ascontiguousarray(a, dtype=np.float64)


def cam_vec(cam) -> np.ndarray:
    """R (9), t (3), fx, fy, cx, cy as float64."""
    return np.concatenate([np.asarray(cam.R, np.float64).reshape(9),
                           np.asarray(cam.t, np.float64).reshape(3),
                           [cam.fx, cam.fy, cam.cx, cam.cy]]).astype(np.float64)


def tiles(cam, cfg: OracleConfig):
    return ((cam.width + cfg.tile_w - 1) // cfg.tile_w,
            (cam.height + cfg.tile_h - 1) // cfg.tile_h)


def num_threads() -> int:
    return int(lib().orc_num_threads())


def set_num_threads(n: int) -> None:
    """OpenMP threads of the oracle's later parallel loops."""
    lib().orc_set_num_threads(int(n))


def sh_basis(deg: int, d, grad: bool = False):
    d = _f64(d)
    nb = (deg + 1) ** 2
    Y = np.zeros(nb)
    dY = np.zeros((nb, 3)) if grad else None
    lib().orc_sh_basis(deg, _p(d), _p(Y), _p(dY))
    return (Y, dY) if grad else Y


def _scene_arrays(scene):
    return (_f64(scene.means), _f64(scene.scales), _f64(scene.quats),
            _f64(scene.opacities), _f64(scene.sh))


def project(scene, cam, cfg: OracleConfig):
    """Projection of every Gaussian (Listing XPR-3DGS, project; with
    cfg.method == "3dgut" the unscented transform of Listing XPR-3DGUT,
    then rec has 21 columns: the 9 of 3DGS, ro, M)."""
    if cfg.method == "3dgut":
        return project_gut(scene, cam, cfg)
    if cfg.method == "linprim":
        return project_lin(scene, cam, cfg)
    m, s, q, o, sh = _scene_arrays(scene)
    n = o.shape[0]
    K = sh.shape[0]
    out = dict(rec=np.zeros((n, 9)), cov=np.zeros((n, 3)), depth=np.zeros(n),
               rect=np.zeros((n, 4), np.int32), tc=np.zeros(n, np.int32),
               radius=np.zeros(n, np.int32), guard=np.zeros(n, np.uint8))
    cv = cam_vec(cam)
    pc = cfg.proj_cfg()
    lib().orc_project(n, _p(m), _p(s), _p(q), _p(o), _p(sh), K, _p(cv), cam.width,
                      cam.height, _p(pc), cfg.tile_w, cfg.tile_h, cfg.sh_degree,
                      _p(out["rec"]), _p(out["cov"]), _p(out["depth"]), _p(out["rect"]),
                      _p(out["tc"]), _p(out["radius"]), _p(out["guard"]))
    return out


def project_gut(scene, cam, cfg: OracleConfig):
    """3DGUT projection (Listing XPR-3DGUT, project)."""
    m, s, q, o, sh = _scene_arrays(scene)
    n = o.shape[0]
    out = dict(rec=np.zeros((n, 21)), cov=np.zeros((n, 3)), depth=np.zeros(n),
               rect=np.zeros((n, 4), np.int32), tc=np.zeros(n, np.int32),
               guard=np.zeros(n, np.uint8))
    lib().orc_project_gut(n, _p(m), _p(s), _p(q), _p(o), _p(sh), _p(cam_vec(cam)), cam.width,
                          cam.height, _p(cfg.gut_cfg()), cfg.tile_w, cfg.tile_h, cfg.sh_degree,
                          _p(out["rec"]), _p(out["cov"]), _p(out["depth"]), _p(out["rect"]),
                          _p(out["tc"]), _p(out["guard"]))
    return out


def project_lin(scene, cam, cfg: OracleConfig):
    """LinPrim projection (Listing XPR-LinPrim, project); rec has 17
    columns: u, v (mu_2D - 1/2), sigma, colour, ex, ey, c0, c1, c2."""
    m, s, q, o, sh = _scene_arrays(scene)
    n = o.shape[0]
    out = dict(rec=np.zeros((n, 17)), depth=np.zeros(n), rect=np.zeros((n, 4), np.int32),
               tc=np.zeros(n, np.int32), guard=np.zeros(n, np.uint8))
    lib().orc_project_lin(n, _p(m), _p(s), _p(q), _p(o), _p(sh), _p(cam_vec(cam)), cam.width,
                          cam.height, _p(cfg.proj_cfg()), cfg.tile_w, cfg.tile_h, cfg.sh_degree,
                          _p(out["rec"]), _p(out["depth"]), _p(out["rect"]), _p(out["tc"]),
                          _p(out["guard"]))
    return out


def lin_chord(rec17, pxy):
    """LinPrim slab intersection: chord length of pixel pxy[k]'s ray in
    record rec17[k] (<= 0: no intersection)."""
    rec17 = _f64(rec17).reshape(-1, 17)
    pxy = np.ascontiguousarray(pxy, np.int32).reshape(-1, 2)
    out = np.zeros(rec17.shape[0])
    lib().orc_lin_chord(rec17.shape[0], _p(rec17), _p(pxy), _p(out))
    return out


def render_fwd_lin(rec, vals, ranges, W: int, H: int, cfg: OracleConfig):
    """LinPrim compositing (Algorithm 1 with the XPR-LinPrim evaluate);
    ``neval`` as for 3DGS."""
    rec = _f64(rec)
    vals = np.ascontiguousarray(vals, np.int32)
    ranges = np.ascontiguousarray(ranges, np.int32)
    out = dict(img=np.zeros((3, H, W)), Tfinal=np.zeros((H, W)),
               ncontrib=np.zeros((H, W), np.int32), nblend=np.zeros((H, W), np.int32),
               guard=np.zeros((H, W), np.uint8), neval=np.zeros((H, W), np.int32))
    lib().orc_render_fwd_lin(W, H, cfg.tile_w, cfg.tile_h, _p(rec), _p(vals), _p(ranges),
                             _p(cfg.render_cfg()), _p(out["img"]), _p(out["Tfinal"]),
                             _p(out["ncontrib"]), _p(out["nblend"]), _p(out["guard"]),
                             _p(out["neval"]))
    return out


def gut_response(rec21, pxy, cam):
    """3DGUT evaluate: the response along the ray of pixel pxy[k] for
    record rec21[k]."""
    rec21 = _f64(rec21).reshape(-1, 21)
    pxy = np.ascontiguousarray(pxy, np.int32).reshape(-1, 2)
    out = np.zeros(rec21.shape[0])
    lib().orc_gut_response(rec21.shape[0], _p(rec21), _p(pxy), _p(cam_vec(cam)), cam.width,
                           cam.height, _p(out))
    return out


def bin_pairs(depth, rect, tc, tiles_x: int, tiles_y: int, cull=None):
    """Binning (section Rasterizer): offsets, I, keys, vals, ranges.

    ``cull`` = (rec, W, H, cfg) applies tile_cull to every replicated pair
    (Listing XPR-3DGS with rec [n][9], XPR-3DGUT with [n][21], XPR-LinPrim
    with [n][17]): culled pairs get the sentinel tile id
    tiles_x*tiles_y and sort last, so the first ``I_kept`` entries of vals
    and keys are the kept lists; ``pair_guard`` flags the pairs whose cull
    decision is in the guard band, in sorted order."""
    depth = _f64(depth)
    rect = np.ascontiguousarray(rect, dtype=np.int32)
    tc = np.ascontiguousarray(tc, dtype=np.int32)
    n = depth.shape[0]
    offsets = np.zeros(n, np.int64)
    I = int(tc.astype(np.int64).sum())
    keys = np.zeros(I, np.uint64)
    vals = np.zeros(I, np.int32)
    ranges = np.zeros((tiles_x * tiles_y, 2), np.int32)
    kept = np.zeros(1, np.int64)
    nguard = np.zeros(1, np.int64)
    pguard = np.zeros(I, np.uint8)
    crec, stride, ext, W, H, tw, th, amin = None, 9, 0, 0, 0, 0, 0, 0.0
    if cull is not None:
        rec, W, H, cfg = cull
        crec = _f64(rec)
        assert crec.shape[0] == n and crec.shape[1] in (9, 17, 21)
        stride = crec.shape[1]
        ext = 1 if cfg.method == "3dgut" else 0
        tw, th, amin = cfg.tile_w, cfg.tile_h, cfg.alpha_min
    got = lib().orc_bin(n, _p(depth), _p(rect), _p(tc), tiles_x, tiles_y, I, _p(offsets),
                        _p(keys), _p(vals), _p(ranges), _p(crec), stride, ext, W, H, tw, th, amin,
                        _p(kept), _p(nguard), _p(pguard))
    assert got == I
    return dict(offsets=offsets, I=I, keys=keys, vals=vals, ranges=ranges,
                I_kept=int(kept[0]), n_guard=int(nguard[0]), pair_guard=pguard)


def tile_cull(rec, txy, W: int, H: int, cfg: OracleConfig):
    """tile_cull of pairs rec[k] x tile txy[k]: keep, power, level, guard.

    3DGS / 3DGUT (Listing XPR-3DGS; rec [m][9]): power is the smallest
    0.5 q over the tile, level log(o / alpha_min). LinPrim (Listing
    XPR-LinPrim; rec [m][17] and cfg.method "linprim"): power is sigma times
    the per-tile chord bound, level -log(1 - alpha_min); kept iff
    power >= level."""
    stride = 17 if cfg.method == "linprim" else 9
    rec = _f64(rec).reshape(-1, stride)
    txy = np.ascontiguousarray(txy, dtype=np.int32).reshape(-1, 2)
    m = rec.shape[0]
    assert txy.shape[0] == m
    keep = np.zeros(m, np.uint8)
    power = np.zeros(m)
    level = np.zeros(m)
    guard = np.zeros(m, np.uint8)
    ext = 1 if cfg.method == "3dgut" else 0
    lib().orc_tile_cull(m, _p(rec), stride, _p(txy), W, H, cfg.tile_w, cfg.tile_h, cfg.alpha_min,
                        ext, _p(keep), _p(power), _p(level), _p(guard))
    return keep.astype(bool), power, level, guard.astype(bool)


def render_fwd(rec, vals, ranges, W: int, H: int, cfg: OracleConfig, cam=None):
    """Compositing (Algorithm 1 with the 3DGS evaluate, or with the 3DGUT
    pixel_info and evaluate when rec has 21 columns; cam is then needed).

    3DGS also returns, per pixel: ``neval`` the list entries it evaluates
    (up to and including the one that stops it, else the whole list);
    ``tsens`` the sensitivity of T_final to a float32 evaluation, in units
    of 2^-24 (1 plus, per blended entry, alpha/(1-alpha) (7 S + 3) + 2 with S
    the sum of the absolute power terms; a clamped alpha adds 2 only);
    ``amb`` [2][H][W] the ambiguous contribution of guard pixels: the
    largest colour change, and the T change, summed over re-walks that each
    invert one guard-band decision (0 elsewhere)."""
    rec = _f64(rec)
    if rec.shape[1] == 21:
        return render_fwd_gut(rec, vals, ranges, cam, cfg)
    if rec.shape[1] == 17:
        return render_fwd_lin(rec, vals, ranges, W, H, cfg)
    vals = np.ascontiguousarray(vals, np.int32)
    ranges = np.ascontiguousarray(ranges, np.int32)
    out = dict(img=np.zeros((3, H, W)), Tfinal=np.zeros((H, W)),
               ncontrib=np.zeros((H, W), np.int32), nblend=np.zeros((H, W), np.int32),
               guard=np.zeros((H, W), np.uint8), neval=np.zeros((H, W), np.int32),
               tsens=np.zeros((H, W)), amb=np.zeros((2, H, W)))
    rc = cfg.render_cfg()
    lib().orc_render_fwd(W, H, cfg.tile_w, cfg.tile_h, _p(rec), _p(vals), _p(ranges), _p(rc),
                         _p(out["img"]), _p(out["Tfinal"]), _p(out["ncontrib"]),
                         _p(out["nblend"]), _p(out["guard"]), _p(out["neval"]),
                         _p(out["tsens"]), _p(out["amb"]))
    return out


def render_fwd_gut(rec, vals, ranges, cam, cfg: OracleConfig):
    """3DGUT compositing (Algorithm 1 with the XPR-3DGUT pixel_info and
    evaluate); ``neval`` as for 3DGS."""
    rec = _f64(rec)
    W, H = cam.width, cam.height
    vals = np.ascontiguousarray(vals, np.int32)
    ranges = np.ascontiguousarray(ranges, np.int32)
    out = dict(img=np.zeros((3, H, W)), Tfinal=np.zeros((H, W)),
               ncontrib=np.zeros((H, W), np.int32), nblend=np.zeros((H, W), np.int32),
               guard=np.zeros((H, W), np.uint8), neval=np.zeros((H, W), np.int32))
    lib().orc_render_fwd_gut(W, H, cfg.tile_w, cfg.tile_h, _p(rec), _p(vals), _p(ranges),
                             _p(cam_vec(cam)), _p(cfg.render_cfg()), _p(out["img"]),
                             _p(out["Tfinal"]), _p(out["ncontrib"]), _p(out["nblend"]),
                             _p(out["guard"]), _p(out["neval"]))
    return out


def render_bwd(rec, vals, ranges, W: int, H: int, cfg: OracleConfig, dimg):
    """dL/d(shader data) [n][9] from dL/dimage [3][H][W]."""
    rec = _f64(rec)
    n = rec.shape[0]
    grad = np.zeros((n, 9))
    rc = cfg.render_cfg()
    dimg = _f64(dimg)
    lib().orc_render_bwd(W, H, cfg.tile_w, cfg.tile_h, n, _p(rec),
                         _p(np.ascontiguousarray(vals, np.int32)),
                         _p(np.ascontiguousarray(ranges, np.int32)), _p(rc), _p(dimg),
                         _p(grad))
    return grad


def project_bwd(scene, cam, cfg: OracleConfig, grad9):
    """Parameter gradients (activated scales/opacity, raw quaternion)."""
    m, s, q, o, sh = _scene_arrays(scene)
    n = o.shape[0]
    K = sh.shape[0]
    g = dict(means=np.zeros((3, n)), scales=np.zeros((3, n)), quats=np.zeros((4, n)),
             opacities=np.zeros(n), sh=np.zeros((K, 3, n)))
    cv = cam_vec(cam)
    pc = cfg.proj_cfg()
    lib().orc_project_bwd(n, _p(m), _p(s), _p(q), _p(o), _p(sh), K, _p(cv), cam.width,
                          cam.height, _p(pc), cfg.tile_w, cfg.tile_h, cfg.sh_degree,
                          _p(_f64(grad9)), _p(g["means"]), _p(g["scales"]), _p(g["quats"]),
                          _p(g["opacities"]), _p(g["sh"]))
    return g


def render(scene, cam, cfg: OracleConfig):
    """Whole forward pipeline in FP64: returns every intermediate."""
    pr = project(scene, cam, cfg)
    tx, ty = tiles(cam, cfg)
    cull = (pr["rec"], cam.width, cam.height, cfg) if cfg.tile_cull else None
    b = bin_pairs(pr["depth"], pr["rect"], pr["tc"], tx, ty, cull)
    f = render_fwd(pr["rec"], b["vals"], b["ranges"], cam.width, cam.height, cfg, cam)
    return dict(proj=pr, bins=b, fwd=f)


def render_bwd_gut(rec, vals, ranges, cam, cfg: OracleConfig, dimg):
    """3DGUT: dL/d(o', r, g, b, ro (3), M (9)) [n][16] from dL/dimage."""
    rec = _f64(rec)
    n = rec.shape[0]
    grad = np.zeros((n, 16))
    lib().orc_render_bwd_gut(cam.width, cam.height, cfg.tile_w, cfg.tile_h, n, _p(rec),
                             _p(np.ascontiguousarray(vals, np.int32)),
                             _p(np.ascontiguousarray(ranges, np.int32)), _p(cam_vec(cam)),
                             _p(cfg.render_cfg()), _p(_f64(dimg)), _p(grad))
    return grad


def project_bwd_gut(scene, cam, cfg: OracleConfig, grad16):
    """3DGUT parameter gradients (activated scales/opacity, raw quaternion)
    from dL/d(o', colour, ro, M) [n][16]."""
    m, s, q, o, sh = _scene_arrays(scene)
    n = o.shape[0]
    K = sh.shape[0]
    g = dict(means=np.zeros((3, n)), scales=np.zeros((3, n)), quats=np.zeros((4, n)),
             opacities=np.zeros(n), sh=np.zeros((K, 3, n)))
    lib().orc_project_bwd_gut(n, _p(m), _p(s), _p(q), _p(o), _p(sh), K, _p(cam_vec(cam)),
                              cam.width, cam.height, _p(cfg.gut_cfg()), cfg.tile_w, cfg.tile_h,
                              cfg.sh_degree, _p(_f64(grad16)), _p(g["means"]), _p(g["scales"]),
                              _p(g["quats"]), _p(g["opacities"]), _p(g["sh"]))
    return g


def render_bwd_lin(rec, vals, ranges, W: int, H: int, cfg: OracleConfig, dimg):
    """LinPrim: dL/d(u, v, sigma, r, g, b, c0 (3), c1 (3), c2 (3), 0) [n][16]
    from dL/dimage."""
    rec = _f64(rec)
    n = rec.shape[0]
    grad = np.zeros((n, 16))
    lib().orc_render_bwd_lin(W, H, cfg.tile_w, cfg.tile_h, n, _p(rec),
                             _p(np.ascontiguousarray(vals, np.int32)),
                             _p(np.ascontiguousarray(ranges, np.int32)), _p(cfg.render_cfg()),
                             _p(_f64(dimg)), _p(grad))
    return grad


def project_bwd_lin(scene, cam, cfg: OracleConfig, grad16):
    """LinPrim parameter gradients (means, half-extent scales, opacity, raw
    quaternion, SH) from the record gradient [n][16]."""
    m, s, q, o, sh = _scene_arrays(scene)
    n = o.shape[0]
    K = sh.shape[0]
    g = dict(means=np.zeros((3, n)), scales=np.zeros((3, n)), quats=np.zeros((4, n)),
             opacities=np.zeros(n), sh=np.zeros((K, 3, n)))
    lib().orc_project_bwd_lin(n, _p(m), _p(s), _p(q), _p(o), _p(sh), K, _p(cam_vec(cam)),
                              cam.width, cam.height, _p(cfg.proj_cfg()), cfg.tile_w, cfg.tile_h,
                              cfg.sh_degree, _p(_f64(grad16)), _p(g["means"]), _p(g["scales"]),
                              _p(g["quats"]), _p(g["opacities"]), _p(g["sh"]))
    return g


def backward(scene, cam, cfg: OracleConfig, dimg, state=None):
    """Analytic gradient of <dimg, image> with respect to the scene (3DGS,
    3DGUT and LinPrim). ``grad9`` (3DGS) or ``grad16`` (3DGUT, LinPrim)
    holds the shader data's gradient."""
    if cfg.method == "linprim":
        st = render(scene, cam, cfg) if state is None else state
        g16 = render_bwd_lin(st["proj"]["rec"], st["bins"]["vals"], st["bins"]["ranges"],
                             cam.width, cam.height, cfg, dimg)
        g = project_bwd_lin(scene, cam, cfg, g16)
        g["grad16"] = g16
        return g
    if cfg.method == "3dgut":
        st = render(scene, cam, cfg) if state is None else state
        g16 = render_bwd_gut(st["proj"]["rec"], st["bins"]["vals"], st["bins"]["ranges"], cam,
                             cfg, dimg)
        g = project_bwd_gut(scene, cam, cfg, g16)
        g["grad16"] = g16
        return g
    if cfg.method != "3dgs":
        raise NotImplementedError(f"unknown method {cfg.method!r}")
    st = render(scene, cam, cfg) if state is None else state
    g9 = render_bwd(st["proj"]["rec"], st["bins"]["vals"], st["bins"]["ranges"],
                    cam.width, cam.height, cfg, dimg)
    g = project_bwd(scene, cam, cfg, g9)
    g["grad9"] = g9
    return g


def l1_loss(image: np.ndarray, target: np.ndarray):
    """The photometric L1 term of the 3DGS training objective (Background
    section), in float64: (mean |image - target|, sign(image - target) / n)
    with sign(0) = 0 and n the number of values."""
    d = np.asarray(image, np.float64) - np.asarray(target, np.float64)
    n = d.size
    return float(np.abs(d).sum() / n), np.sign(d) / n
