"""Pins of the oracle's opacity-aware extents (compute_extents of the listing
"Implementation of XPR-3DGS" takes the opacity): the half-widths of the
ellipse where o G = alpha_min, against the closed form of an on-axis
isotropic Gaussian and against a dense parametrisation of the ellipse's
boundary; every pixel that passes the alpha gate lies in the rect; the image
is then independent of the tile size at any opacity and equals the per-pixel
brute force with unbounded support; the analytic gradient matches autograd
of the brute force."""
import math

import numpy as np
import pytest
import torch

import oracle
import oracle.brute as brute
from helpers import axis_camera, hand_scene
from synth import camera_look_at, scene_clusters

A_MIN = 1.0 / 255.0


def _cfg(**kw):
    kw.setdefault("sh_degree", 0)
    kw.setdefault("opacity_extents", True)
    return oracle.OracleConfig(**kw)


@pytest.mark.parametrize("o", [0.995, 0.6, 0.1, 0.01])
def test_on_axis_isotropic_rect(o):
    W, H, f, Z, s = 257, 181, 300.0, 4.0, 0.05
    cam = axis_camera(W, H, f=f)
    sc = hand_scene([[0.013, -0.021, Z]], [s, s, s], opac=o)
    pr = oracle.project(sc, cam, _cfg())
    s32, o32 = float(np.float32(s)), float(np.float32(o))
    var = (f * s32 / Z) ** 2 + 0.3
    u, v = pr["rec"][0, 0], pr["rec"][0, 1]
    e = math.sqrt(2 * math.log(o32 / A_MIN) * var)
    want = [math.floor((u - e) / 16), math.floor((v - e) / 16),
            math.floor((u + e) / 16) + 1, math.floor((v + e) / 16) + 1]
    want = [min(max(w, 0), lim) for w, lim in zip(want, [17, 12, 17, 12])]
    assert list(pr["rect"][0]) == want
    assert pr["tc"][0] == (want[2] - want[0]) * (want[3] - want[1])
    # against the 3-sigma rule: wider above o = e^4.5 / 255, narrower below
    r3 = math.ceil(3 * math.sqrt(var))
    assert (e > r3) == (o32 > math.exp(4.5) / 255 and e > r3)


def test_extents_are_the_alpha_ellipse_bounding_box():
    sc = scene_clusters(400, seed=2, n_clusters=3, box=1.0, lo=0.01, hi=0.3)
    cam = camera_look_at((0.3, -0.2, -4.0), 300, 200)
    cfg = _cfg(sh_degree=3)
    pr = oracle.project(sc, cam, cfg)
    t = np.linspace(0, 2 * np.pi, 200_001)
    circ = np.stack([np.cos(t), np.sin(t)])
    n = 0
    for i in np.nonzero(pr["tc"] > 0)[0][:60]:
        a, b, c = pr["cov"][i]
        lvl = 2 * math.log(sc.opacities[i] / np.float32(A_MIN))
        L = np.linalg.cholesky(np.array([[a, b], [b, c]]))
        pts = math.sqrt(lvl) * (L @ circ)          # the ellipse d^T cov^-1 d = lvl
        ex, ey = np.abs(pts[0]).max(), np.abs(pts[1]).max()
        u, v = pr["rec"][i, :2]
        x0, y0, x1, y1 = pr["rect"][i]
        # the rect is the tiles of [u - ex, u + ex] x [v - ey, v + ey] (the
        # sampled maximum is within 1e-9 of the true one)
        for lo, hi, m, lim in ((x0, x1, u, ex), (y0, y1, v, ey)):
            assert lo <= max(math.floor((m - lim * (1 + 1e-9)) / 16), 0)
            assert hi >= math.floor((m + lim * (1 - 1e-9)) / 16) + 1 or hi == (
                cam.width + 15) // 16 or hi == (cam.height + 15) // 16
        n += 1
    assert n > 30


def test_every_passing_pixel_is_in_the_rect():
    sc = scene_clusters(300, seed=3, n_clusters=3, box=1.0, lo=0.01, hi=0.3)
    sc.opacities[:] = np.float32(0.97)
    cam = camera_look_at((0.2, 0.1, -4.0), 120, 90)
    ys, xs = np.mgrid[0:cam.height, 0:cam.width]
    outside = {}
    for mode in (True, False):
        pr = oracle.project(sc, cam, _cfg(opacity_extents=mode))
        cnt = 0
        for i in np.nonzero(pr["tc"] > 0)[0]:
            r = pr["rec"][i]
            dx, dy = xs - r[0], ys - r[1]
            P = r[2] * dx * dx + r[3] * dx * dy + r[4] * dy * dy
            lit = (P <= 0) & (r[5] * np.exp(P) >= A_MIN)
            x0, y0, x1, y1 = pr["rect"][i]
            inside = (xs // 16 >= x0) & (xs // 16 < x1) & (ys // 16 >= y0) & (ys // 16 < y1)
            cnt += int((lit & ~inside).sum())
        outside[mode] = cnt
    assert outside[True] == 0
    assert outside[False] > 0  # the 3-sigma box misses pixels of opaque Gaussians


@pytest.mark.parametrize("opaque", [False, True])
def test_tile_size_invariance_at_any_opacity(opaque):
    sc = scene_clusters(500, seed=4, n_clusters=4, box=1.0, lo=0.005, hi=0.3)
    if opaque:
        sc.opacities[:] = np.float32(0.98)
    cam = camera_look_at((0.2, 0.1, -4.0), 70, 52)
    imgs = [oracle.render(sc, cam, _cfg(sh_degree=3, tile_w=t, tile_h=t))["fwd"]["img"]
            for t in (8, 16, 32)]
    np.testing.assert_array_equal(imgs[0], imgs[1])
    np.testing.assert_array_equal(imgs[0], imgs[2])
    # unbounded support: one tile covering the whole image
    ib, _ = brute.render(sc, cam, _cfg(sh_degree=3, tile_w=1024, tile_h=1024,
                                       opacity_extents=False))
    np.testing.assert_allclose(imgs[1], ib, atol=1e-13)
    if opaque:
        # the 3-sigma rect cuts opaque Gaussians off at tile-dependent places
        plain = [oracle.render(sc, cam, _cfg(sh_degree=3, tile_w=t, tile_h=t,
                                             opacity_extents=False))["fwd"]["img"]
                 for t in (8, 32)]
        assert not np.array_equal(plain[0], plain[1])


@pytest.mark.parametrize("tile", [8, 16])
def test_brute_force_equals_tiled(tile):
    sc = scene_clusters(150, seed=6, n_clusters=3, box=1.0, lo=0.01, hi=0.3)
    cam = camera_look_at((0.5, -0.3, -4.5), 50, 37)
    cfg = _cfg(sh_degree=3, tile_w=tile, tile_h=tile, bg=(0.1, 0.2, 0.3))
    st = oracle.render(sc, cam, cfg)
    ib, Tb = brute.render(sc, cam, cfg)
    np.testing.assert_allclose(st["fwd"]["img"], ib, atol=1e-13)
    np.testing.assert_allclose(st["fwd"]["Tfinal"], Tb, atol=1e-13)


def test_gradient_matches_autograd_of_brute_force():
    sc = scene_clusters(40, seed=7, n_clusters=2, box=0.8, lo=0.02, hi=0.25)
    cam = camera_look_at((0.2, 0.3, -4.0), 40, 30)
    cfg = _cfg(sh_degree=3, tile_w=8, tile_h=8)
    rng = np.random.default_rng(0)
    dimg = rng.normal(size=(3, cam.height, cam.width))
    g = oracle.backward(sc, cam, cfg, dimg)
    ts = brute.scene_tensors(sc, requires_grad=True)
    img, _ = brute.render_torch(*ts, cam, cfg)
    (img * torch.as_tensor(dimg)).sum().backward()
    ref = {"means": ts[0].grad.numpy().T, "scales": ts[1].grad.numpy().T,
           "quats": ts[2].grad.numpy().T, "opacities": ts[3].grad.numpy(),
           "sh": np.transpose(ts[4].grad.numpy(), (1, 2, 0))}
    for f in ("means", "scales", "quats", "opacities", "sh"):
        scale = max(np.abs(ref[f]).max(), 1e-12)
        assert np.abs(g[f] - ref[f]).max() <= 1e-7 * scale, f
