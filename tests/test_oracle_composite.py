"""Pins of the oracle's compositing (Algorithm 1 with the 3DGS evaluate and
the blending of the Background section): closed forms, invariants,
tile-size invariance and the per-pixel brute force."""
import json
import math
import os

import numpy as np
import pytest

import oracle
import oracle.brute as brute
from helpers import axis_camera, hand_scene
from synth import camera_look_at, scene_clusters, scene_uniform_cube

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def _cfg(**kw):
    kw.setdefault("sh_degree", 0)
    return oracle.OracleConfig(**kw)


def test_single_gaussian_closed_form():
    # (a) image(p) = c * min(.99, o exp(-|p - mu|^2 / (2 var))) where that is
    # >= 1/255 and tile(p) lies in the rect, else background.
    W, H, f, Z, s, o = 65, 49, 200.0, 4.0, 0.06, 0.8
    cam = axis_camera(W, H, f=f)
    cfg = _cfg()
    sc = hand_scene([[0, 0, Z]], [s, s, s], opac=o, rgb=[0.9, 0.4, 0.2])
    st = oracle.render(sc, cam, cfg)
    s32, o32 = float(np.float32(s)), float(np.float32(o))
    var = (f * s32 / Z) ** 2 + 0.3
    u, v = W / 2 - 0.5, H / 2 - 0.5
    col = st["proj"]["rec"][0, 6:]
    x0, y0, x1, y1 = st["proj"]["rect"][0]
    ys, xs = np.mgrid[0:H, 0:W]
    a = np.minimum(0.99, o32 * np.exp(-((xs - u) ** 2 + (ys - v) ** 2) / (2 * var)))
    inside = (xs // 16 >= x0) & (xs // 16 < x1) & (ys // 16 >= y0) & (ys // 16 < y1)
    lit = inside & (a >= 1 / 255)
    exp = np.where(lit[None], col[:, None, None] * a[None], 0.0)
    np.testing.assert_allclose(st["fwd"]["img"], exp, atol=1e-14)
    assert int((st["fwd"]["nblend"] > 0).sum()) == int(lit.sum())
    np.testing.assert_array_equal(st["fwd"]["ncontrib"], lit.astype(np.int32))


@pytest.mark.parametrize("case", json.load(open(os.path.join(GOLDEN, "stop_rule.json")))["cases"],
                         ids=lambda c: f"o{c['opacity']}")
def test_stop_rule_on_axis_stack(case):
    # (b) K Gaussians on the axis at depths 1..K; at the axis pixel a_i = o.
    W, H, K = 33, 31, 40
    o = case["opacity"]
    cam = axis_camera(W, H, f=40.0)
    cfg = _cfg()
    means = [[0, 0, 1.0 + k] for k in range(K)]
    sc = hand_scene(means, [0.01, 0.01, 0.01], opac=o, rgb=[0.7, 0.3, 0.5])
    st = oracle.render(sc, cam, cfg)
    px, py = (W - 1) // 2, (H - 1) // 2
    o32 = float(np.float32(o))
    k = case["blended"]
    assert st["fwd"]["nblend"][py, px] == k
    assert st["fwd"]["ncontrib"][py, px] == k
    assert (1 - o32) ** k >= 1e-4 > (1 - o32) ** (k + 1)
    col = st["proj"]["rec"][0, 6:]
    np.testing.assert_allclose(st["fwd"]["img"][:, py, px], col * (1 - (1 - o32) ** k), rtol=1e-13)
    assert st["fwd"]["Tfinal"][py, px] == pytest.approx((1 - o32) ** k, rel=1e-13)


def test_two_gaussian_order_closed_form():
    # (e) C = c1 a1 + c2 a2 (1 - a1) for a front Gaussian 1 and back Gaussian 2.
    W, H = 41, 41
    cam = axis_camera(W, H, f=80.0)
    cfg = _cfg()
    sc = hand_scene([[0.02, 0.0, 3.0], [-0.01, 0.02, 5.0]], [0.08, 0.08, 0.08],
                    opac=[0.6, 0.7], rgb=[[1.0, 0.0, 0.2], [0.0, 1.0, 0.4]])
    st = oracle.render(sc, cam, cfg)
    rec = st["proj"]["rec"]
    for (px, py) in [(20, 20), (22, 19), (18, 23)]:
        al = []
        for g in range(2):
            dx, dy = px - rec[g, 0], py - rec[g, 1]
            P = rec[g, 2] * dx * dx + rec[g, 3] * dx * dy + rec[g, 4] * dy * dy
            al.append(min(0.99, rec[g, 5] * math.exp(P)))
        exp = rec[0, 6:] * al[0] + rec[1, 6:] * al[1] * (1 - al[0])
        np.testing.assert_allclose(st["fwd"]["img"][:, py, px], exp, rtol=1e-13)


def _white_scene(n, seed):
    sc = scene_uniform_cube(n, seed)
    sc.sh[0] = np.float32(0.5 / (0.5 / math.sqrt(math.pi)))  # colour exactly ~1
    return sc


def test_telescoping_white():
    # (c) all colours 1, background 0: C = 1 - T_final at every pixel.
    sc = _white_scene(400, 4)
    cam = camera_look_at((0.0, 0.0, -4.0), 64, 48)
    cfg = _cfg()
    st = oracle.render(sc, cam, cfg)
    col = st["proj"]["rec"][:, 6:]
    c = float(col[st["proj"]["tc"] > 0][0, 0])
    assert np.allclose(col[st["proj"]["tc"] > 0], c, rtol=0, atol=0)
    np.testing.assert_allclose(st["fwd"]["img"] / c, np.broadcast_to(1 - st["fwd"]["Tfinal"], (3, 48, 64)),
                               atol=1e-13)


def test_bounds_and_invariants():
    # (d) 0 <= C_k <= (1 - T_final) max c_k; T_final in [1e-4, 1].
    sc = scene_clusters(3000, seed=1, n_clusters=8, box=1.0)
    cam = camera_look_at((0.0, 1.0, -5.0), 80, 64)
    cfg = _cfg(sh_degree=3)
    st = oracle.render(sc, cam, cfg)
    T = st["fwd"]["Tfinal"]
    assert T.min() >= 1e-4 and T.max() <= 1.0
    cmax = st["proj"]["rec"][st["proj"]["tc"] > 0, 6:].max(0)
    img = st["fwd"]["img"]
    assert img.min() >= 0
    assert np.all(img <= (1 - T)[None] * cmax[:, None, None] + 1e-12)


def test_tile_size_invariance_low_opacity():
    # (f) with every o < e^4.5/255 the image does not depend on the tile size
    # (alpha >= 1/255 then forces Mahalanobis^2 < 9, inside the 3-sigma rect).
    sc = scene_uniform_cube(600, 3)
    sc.opacities = np.minimum(sc.opacities, np.float32(0.35))
    cam = camera_look_at((0.2, 0.1, -4.0), 70, 52)
    imgs = []
    for t in (8, 16, 32):
        imgs.append(oracle.render(sc, cam, _cfg(tile_w=t, tile_h=t))["fwd"]["img"])
    np.testing.assert_array_equal(imgs[0], imgs[1])
    np.testing.assert_array_equal(imgs[0], imgs[2])
    ib, _ = brute.render(sc, cam, _cfg(tile_w=1024, tile_h=1024))
    np.testing.assert_allclose(imgs[0], ib, atol=1e-13)


@pytest.mark.parametrize("seed,tile", [(0, 16), (1, 8), (2, 16)])
def test_brute_force_equals_tiled(seed, tile):
    # (g) per-pixel brute force (no pairs, no sort, no ranges) == tiled oracle.
    sc = scene_clusters(150, seed=seed, n_clusters=3, box=1.0, lo=0.01, hi=0.3)
    cam = camera_look_at((0.5, -0.3, -4.5), 50, 37)
    cfg = _cfg(sh_degree=3, tile_w=tile, tile_h=tile, bg=(0.1, 0.2, 0.3))
    st = oracle.render(sc, cam, cfg)
    ib, Tb = brute.render(sc, cam, cfg)
    np.testing.assert_allclose(st["fwd"]["img"], ib, atol=1e-13)
    np.testing.assert_allclose(st["fwd"]["Tfinal"], Tb, atol=1e-13)
