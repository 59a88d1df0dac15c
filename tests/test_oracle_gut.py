"""Pins of the oracle's 3DGUT path (Listing "Implementation of XPR-3DGUT",
forward): the unscented transform against closed forms (exact for a planar
Gaussian facing the camera, by hand for one stretched along the optical
axis, and close to the independently pinned EWA projection for small
Gaussians), the ray response against the world-space Mahalanobis distance of
the ray and a bounded scalar minimiser, the pixel ray through the pixel
centre, a single-Gaussian image in closed form, and the per-pixel brute
force (no pairs, no sort) equal to the tiled oracle."""
import math

import numpy as np
import pytest
from scipy.optimize import minimize_scalar

import oracle
import oracle.brute as brute
from helpers import axis_camera, hand_scene, quat_z, random_rotation
from synth import camera_look_at, scene_clusters

Y00 = 0.5 / math.sqrt(math.pi)


def _cfg(**kw):
    kw.setdefault("sh_degree", 0)
    kw.setdefault("method", "3dgut")
    return oracle.OracleConfig(**kw)


def _f32(x):
    return float(np.float32(x))


def test_planar_gaussian_facing_the_camera_is_exact():
    # all sigma points at one depth: the projection is affine there, so the
    # transform is exact: mean = projection of mu, cov = (f/z)^2 R2 S2^2 R2^T
    W, H, f, z0 = 200, 150, 180.0, 5.0
    cam = axis_camera(W, H, f=f)
    th = 0.7
    sx, sy = 0.04, 0.015
    sc = hand_scene([[0.31, -0.22, z0]], [[sx, sy, 1e-9]], quats=[quat_z(th)], opac=0.8)
    pr = oracle.project(sc, cam, _cfg())
    mu = sc.means[:, 0].astype(np.float64)
    s = sc.scales[:, 0].astype(np.float64)
    q = sc.quats[:, 0].astype(np.float64)
    ang = 2 * math.atan2(q[3], q[0])
    R2 = np.array([[math.cos(ang), -math.sin(ang)], [math.sin(ang), math.cos(ang)]])
    k = f / mu[2]
    cov = k * k * R2 @ np.diag(s[:2] ** 2) @ R2.T
    u = f * mu[0] / mu[2] + W / 2 - 0.5
    v = f * mu[1] / mu[2] + H / 2 - 0.5
    np.testing.assert_allclose(pr["rec"][0, :2], [u, v], rtol=0, atol=1e-12)
    np.testing.assert_allclose(pr["cov"][0], [cov[0, 0] + 0.3, cov[0, 1], cov[1, 1] + 0.3],
                               rtol=1e-12, atol=1e-12)


def test_stretch_along_the_optical_axis_by_hand():
    # R = I, mu off-axis: four sigma points share the depth z0, two sit at
    # z0 +- sqrt(3) sz; mean weights 0 (centre) and 1/6, covariance weights
    # 2 (centre) and 1/6
    W, H, f = 160, 120, 150.0
    cam = axis_camera(W, H, f=f)
    sc = hand_scene([[0.5, -0.3, 4.0]], [[0.05, 0.02, 0.4]], opac=0.7)
    pr = oracle.project(sc, cam, _cfg())
    x0, y0, z0 = sc.means[:, 0].astype(np.float64)
    sx, sy, sz = sc.scales[:, 0].astype(np.float64)
    r3 = math.sqrt(3)
    pts = [(x0, y0, z0), (x0 + r3 * sx, y0, z0), (x0 - r3 * sx, y0, z0), (x0, y0 + r3 * sy, z0),
           (x0, y0 - r3 * sy, z0), (x0, y0, z0 + r3 * sz), (x0, y0, z0 - r3 * sz)]
    P = np.array([[f * x / z + W / 2, f * y / z + H / 2] for x, y, z in pts])
    wm = np.array([0] + [1 / 6] * 6)
    wc = np.array([2] + [1 / 6] * 6)
    m = wm @ P
    D = P - m
    cov = (wc[:, None, None] * D[:, :, None] * D[:, None, :]).sum(0)
    np.testing.assert_allclose(pr["rec"][0, :2], m - 0.5, rtol=0, atol=1e-10)
    np.testing.assert_allclose(pr["cov"][0], [cov[0, 0] + 0.3, cov[0, 1], cov[1, 1] + 0.3],
                               rtol=1e-12)
    det0 = cov[0, 0] * cov[1, 1] - cov[0, 1] ** 2
    det = (cov[0, 0] + 0.3) * (cov[1, 1] + 0.3) - cov[0, 1] ** 2
    assert pr["rec"][0, 5] == pytest.approx(_f32(0.7) * math.sqrt(det0 / det), rel=1e-12)


def test_small_gaussians_agree_with_ewa():
    sc = scene_clusters(400, seed=2, n_clusters=3, box=1.0, lo=0.001, hi=0.004)
    cam = camera_look_at((0.2, 0.1, -5.0), 320, 240)
    g = oracle.project(sc, cam, _cfg(sh_degree=3))
    e = oracle.project(sc, cam, oracle.OracleConfig(sh_degree=3))
    m = (g["tc"] > 0) & (e["tc"] > 0)
    assert m.sum() > 300
    # first order agreement: the second-order terms are (s / z)^2 ~ 1e-6 of f
    assert np.abs(g["rec"][m, :2] - e["rec"][m, :2]).max() < 2e-3
    cg, ce = g["cov"][m] - [0.3, 0, 0.3], e["cov"][m] - [0.3, 0, 0.3]
    scale = np.maximum(cg[:, 0], cg[:, 2])[:, None]
    assert (np.abs(cg - ce) / scale).max() < 1e-2


def _world_d2(mu, Rq, s, cp, rd):
    Sinv = Rq @ np.diag(1 / s ** 2) @ Rq.T
    D = cp - mu
    return D @ Sinv @ D - (D @ Sinv @ rd) ** 2 / (rd @ Sinv @ rd)


def _ray(cam, px, py):
    d = np.array([(px + 0.5 - cam.cx) / cam.fx, (py + 0.5 - cam.cy) / cam.fy, 1.0])
    return np.asarray(cam.R).T @ (d / np.linalg.norm(d))


def _quat_to_rot(q):
    w, x, y, z = q / np.linalg.norm(q)
    return np.array([[1 - 2 * (y * y + z * z), 2 * (x * y - w * z), 2 * (x * z + w * y)],
                     [2 * (x * y + w * z), 1 - 2 * (x * x + z * z), 2 * (y * z - w * x)],
                     [2 * (x * z - w * y), 2 * (y * z + w * x), 1 - 2 * (x * x + y * y)]])


def test_response_is_the_mahalanobis_distance_of_the_ray():
    rng = np.random.default_rng(3)
    sc = scene_clusters(60, seed=3, n_clusters=2, box=0.8, lo=0.02, hi=0.3)
    cam = camera_look_at((0.4, -0.3, -4.0), 90, 70)
    pr = oracle.project(sc, cam, _cfg(sh_degree=3))
    cp = -np.asarray(cam.R).T @ np.asarray(cam.t)
    idx = np.repeat(np.arange(sc.n), 5)
    pxy = np.stack([rng.integers(0, cam.width, idx.size), rng.integers(0, cam.height, idx.size)], 1)
    got = oracle.gut_response(pr["rec"][idx], pxy, cam)
    for k, i in enumerate(idx):
        mu = sc.means[:, i].astype(np.float64)
        s = sc.scales[:, i].astype(np.float64)
        Rq = _quat_to_rot(sc.quats[:, i].astype(np.float64))
        rd = _ray(cam, *pxy[k])
        d2 = _world_d2(mu, Rq, s, cp, rd)
        assert got[k] == pytest.approx(math.exp(-0.5 * d2), rel=1e-9, abs=1e-300)
        if k % 25 == 0:  # and against a scalar minimiser along the ray
            Sinv = Rq @ np.diag(1 / s ** 2) @ Rq.T
            fn = lambda t: (cp + t * rd - mu) @ Sinv @ (cp + t * rd - mu)
            r = minimize_scalar(fn, bracket=(0.0, 10.0), tol=1e-12)
            assert d2 == pytest.approx(r.fun, rel=1e-6, abs=1e-9)


def test_pixel_ray_goes_through_the_pixel_centre():
    # an isotropic Gaussian centred on the ray of pixel (px, py) responds 1 there
    cam = camera_look_at((0.5, 0.2, -3.0), 64, 48)
    R = np.asarray(cam.R)
    cp = -R.T @ np.asarray(cam.t)
    for px, py in [(0, 0), (13, 30), (63, 47)]:
        mu = cp + 2.5 * _ray(cam, px, py)
        sc = hand_scene([mu], [0.05, 0.05, 0.05], opac=0.5)
        rec = oracle.project(sc, cam, _cfg())["rec"]
        ref = oracle.gut_response(rec, [[px, py]], cam)[0]
        assert ref == pytest.approx(1.0, abs=1e-12)
        nb = oracle.gut_response(rec, [[px + 1, py]], cam)[0]
        assert nb < 1.0 - 1e-3


def test_single_gaussian_image_closed_form():
    # on-axis, unrotated: the UT covariance is (f s / z)^2 I exactly (the
    # depth sigma points project onto the centre), so o' is known in closed
    # form; image(p) = c min(.99, o' response(p)) where response > 0.0113,
    # alpha >= 1/255 and the pixel's tile is in the rect
    W, H, f, Z, s, sz, o = 61, 47, 120.0, 4.0, 0.06, 0.09, 0.8
    cam = axis_camera(W, H, f=f)
    sc = hand_scene([[0, 0, Z]], [[s, s, sz]], opac=o, rgb=[0.9, 0.4, 0.2])
    cfg = _cfg()
    st = oracle.render(sc, cam, cfg)
    s32, sz32, o32 = _f32(s), _f32(sz), _f32(o)
    k2 = (f * s32 / Z) ** 2
    o2 = o32 * k2 / (k2 + 0.3)
    assert st["proj"]["rec"][0, 5] == pytest.approx(o2, rel=1e-12)
    col = st["proj"]["rec"][0, 6:9]
    x0, y0, x1, y1 = st["proj"]["rect"][0]
    cp = np.zeros(3)
    mu = np.array([0, 0, _f32(Z)])
    exp = np.zeros((3, H, W))
    for py in range(H):
        for px in range(W):
            d2 = _world_d2(mu, np.eye(3), np.array([s32, s32, sz32]), cp, _ray(cam, px, py))
            resp = math.exp(-0.5 * d2)
            a = min(0.99, o2 * resp)
            inside = x0 <= px // 16 < x1 and y0 <= py // 16 < y1
            if inside and resp > 0.0113 and a >= 1 / 255:
                exp[:, py, px] = col * a
    np.testing.assert_allclose(st["fwd"]["img"], exp, atol=1e-12)
    assert (exp > 0).sum() > 100


@pytest.mark.parametrize("seed,tile,ext", [(0, 16, False), (1, 8, False), (2, 16, True)])
def test_brute_force_equals_tiled(seed, tile, ext):
    sc = scene_clusters(150, seed=seed, n_clusters=3, box=1.0, lo=0.01, hi=0.3)
    cam = camera_look_at((0.5, -0.3, -4.5), 50, 37)
    cfg = _cfg(sh_degree=3, tile_w=tile, tile_h=tile, bg=(0.1, 0.2, 0.3), opacity_extents=ext)
    st = oracle.render(sc, cam, cfg)
    ib, Tb = brute.render_gut(sc, cam, cfg)
    np.testing.assert_allclose(st["fwd"]["img"], ib, atol=1e-13)
    np.testing.assert_allclose(st["fwd"]["Tfinal"], Tb, atol=1e-13)


def test_cull_tile_bounds_extended_by_one_pixel():
    # isotropic conic: the smallest power is a squared distance to the box
    # [x tw, min(x tw + tw - 1, W - 1) + 1] (likewise y)
    rng = np.random.default_rng(5)
    W, H = 100, 70
    recs, txy, exp = [], [], []
    for _ in range(300):
        u, v = rng.uniform(-20, W + 20), rng.uniform(-20, H + 20)
        a = math.exp(rng.uniform(-6, 0.5))
        tx, ty = rng.integers(0, 7), rng.integers(0, 5)
        x0, y0 = tx * 16, ty * 16
        x1, y1 = min(x0 + 15, W - 1) + 1, min(y0 + 15, H - 1) + 1
        d2 = max(x0 - u, 0, u - x1) ** 2 + max(y0 - v, 0, v - y1) ** 2
        recs.append([u, v, -0.5 * a, 0.0, -0.5 * a, 0.6] + [0.5] * 3)
        txy.append((tx, ty))
        exp.append(0.5 * a * d2)
    _, power, _, _ = oracle.tile_cull(np.array(recs), np.array(txy), W, H, _cfg())
    np.testing.assert_allclose(power, exp, rtol=1e-12, atol=1e-300)
