"""Pins of the oracle's LinPrim path (Listing "Implementation of
XPR-LinPrim", forward): the linear map A against finite differences of the
pinhole projection and of the Euclidean distance, the rows of A^-1 and the
chord of an axis-aligned on-axis octahedron in closed form, Beer-Lambert
through the centre along the shortest axis (0.99 o), the slab chord against
scipy's linear-programming solver for general octahedra, and the per-pixel
brute force equal to the tiled oracle."""
import math

import numpy as np
import pytest
from scipy.optimize import linprog

import oracle
import oracle.brute as brute
from helpers import axis_camera, hand_scene
from synth import camera_look_at, scene_clusters


def _cfg(**kw):
    kw.setdefault("sh_degree", 0)
    kw.setdefault("method", "linprim")
    return oracle.OracleConfig(**kw)


def _f32(x):
    return float(np.float32(x))


def test_on_axis_octahedron_closed_form():
    W, H, f, z0 = 81, 61, 100.0, 4.0
    sx, sy, sz, o = 0.3, 0.2, 0.1, 0.7
    cam = axis_camera(W, H, f=f)
    sc = hand_scene([[0, 0, z0]], [[sx, sy, sz]], opac=o, rgb=[0.9, 0.5, 0.1])
    pr = oracle.project(sc, cam, _cfg())
    sx, sy, sz, o = _f32(sx), _f32(sy), _f32(sz), _f32(o)
    r = pr["rec"][0]
    np.testing.assert_allclose(r[:2], [W / 2 - 0.5, H / 2 - 0.5], atol=1e-12)
    np.testing.assert_allclose(r[6:8], [f * sx / z0, f * sy / z0], rtol=1e-12)
    c = r[8:17].reshape(3, 3)
    np.testing.assert_allclose(c, np.diag([z0 / (f * sx), z0 / (f * sy), 1 / sz]), atol=1e-12)
    sigma = -math.log1p(-0.99 * o) / (2 * sz)
    assert r[2] == pytest.approx(sigma, rel=1e-12)
    assert pr["depth"][0] == pytest.approx(z0)
    # chord 2 sz (1 - |dx| z0 / (f sx) - |dy| z0 / (f sy)), alpha by Beer-Lambert
    rng = np.random.default_rng(0)
    pxy = np.stack([rng.integers(0, W, 200), rng.integers(0, H, 200)], 1)
    got = oracle.lin_chord(np.repeat(r[None], len(pxy), 0), pxy)
    for k, (px, py) in enumerate(pxy):
        a = abs(px + 0.5 - W / 2) * z0 / (f * sx) + abs(py + 0.5 - H / 2) * z0 / (f * sy)
        want = 2 * sz * (1 - a)
        if want > 0:
            assert got[k] == pytest.approx(want, rel=1e-12, abs=1e-15)
        else:
            assert got[k] <= 1e-15
    # through the centre along the shortest axis: alpha = 0.99 o
    st = oracle.render(sc, cam, _cfg())
    ctr = st["fwd"]["img"][:, 30, 40] / np.array(st["proj"]["rec"][0, 3:6])
    assert ctr[0] == pytest.approx(0.99 * o, rel=1e-12)


def test_linear_map_rows_are_the_derivatives():
    # columns of A: (d pixel / d e_k, d |mu_c| / d e_k) for e_k = s_k R e_k,
    # checked by central differences of the exact maps
    sc = scene_clusters(30, seed=1, n_clusters=2, box=0.8, lo=0.01, hi=0.1)
    cam = camera_look_at((0.4, -0.3, -4.0), 90, 70)
    pr = oracle.project(sc, cam, _cfg())
    Rw, tw = np.asarray(cam.R), np.asarray(cam.t)
    for i in range(sc.n):
        if pr["tc"][i] == 0:
            continue
        c = pr["rec"][i, 8:17].reshape(3, 3)
        A = np.linalg.inv(c)
        mu = sc.means[:, i].astype(np.float64)
        q = sc.quats[:, i].astype(np.float64)
        q = q / np.linalg.norm(q)
        w, x, y, z = q
        Rq = np.array([[1 - 2 * (y * y + z * z), 2 * (x * y - w * z), 2 * (x * z + w * y)],
                       [2 * (x * y + w * z), 1 - 2 * (x * x + z * z), 2 * (y * z - w * x)],
                       [2 * (x * z - w * y), 2 * (y * z + w * x), 1 - 2 * (x * x + y * y)]])
        s = sc.scales[:, i].astype(np.float64)

        def f(p):
            pc = Rw @ p + tw
            return np.array([cam.fx * pc[0] / pc[2], cam.fy * pc[1] / pc[2], np.linalg.norm(pc)])
        for k in range(3):
            e = Rq[:, k] * s[k]
            h = 1e-5
            fd = (f(mu + h * e) - f(mu - h * e)) / (2 * h)
            np.testing.assert_allclose(A[:, k], fd, rtol=1e-6, atol=1e-8)
        # the sort depth is the Euclidean distance that tau measures
        assert pr["depth"][i] == pytest.approx(f(mu)[2], rel=1e-13)


def test_chord_matches_linear_programming():
    sc = scene_clusters(40, seed=2, n_clusters=2, box=0.8, lo=0.02, hi=0.2)
    cam = camera_look_at((0.2, 0.3, -3.5), 80, 60)
    pr = oracle.project(sc, cam, _cfg())
    rng = np.random.default_rng(2)
    checked = 0
    for i in np.nonzero(pr["tc"] > 0)[0]:
        r = pr["rec"][i]
        c = r[8:17].reshape(3, 3)
        for _ in range(12):
            px = int(np.clip(rng.normal(r[0], r[6] * 0.6), 0, cam.width - 1))
            py = int(np.clip(rng.normal(r[1], r[7] * 0.6), 0, cam.height - 1))
            dx, dy = px - r[0], py - r[1]
            # variables (tau, t0, t1, t2): -t_k <= c_k . (dx, dy, tau) <= t_k, sum t <= 1
            A_ub, b_ub = [], []
            for k in range(3):
                a0 = c[k, 0] * dx + c[k, 1] * dy
                row = [c[k, 2], 0, 0, 0]
                row[1 + k] = -1
                A_ub.append(row); b_ub.append(-a0)
                row = [-c[k, 2], 0, 0, 0]
                row[1 + k] = -1
                A_ub.append(row); b_ub.append(a0)
            A_ub.append([0, 1, 1, 1]); b_ub.append(1)
            bounds = [(None, None), (0, None), (0, None), (0, None)]
            lo = linprog([1, 0, 0, 0], A_ub=A_ub, b_ub=b_ub, bounds=bounds, method="highs")
            hi = linprog([-1, 0, 0, 0], A_ub=A_ub, b_ub=b_ub, bounds=bounds, method="highs")
            got = oracle.lin_chord(r[None], [[px, py]])[0]
            if lo.status == 2:  # infeasible: the ray misses
                assert got <= 1e-9
                continue
            want = hi.x[0] - lo.x[0]
            scale = max(abs(lo.x[0]), abs(hi.x[0]), 1e-12)
            assert got == pytest.approx(want, abs=1e-7 * scale), (i, px, py)
            checked += 1
    assert checked > 100


@pytest.mark.parametrize("seed,tile", [(0, 16), (1, 8)])
def test_brute_force_equals_tiled(seed, tile):
    sc = scene_clusters(150, seed=seed, n_clusters=3, box=1.0, lo=0.01, hi=0.25)
    cam = camera_look_at((0.5, -0.3, -4.5), 50, 37)
    cfg = _cfg(sh_degree=3, tile_w=tile, tile_h=tile, bg=(0.1, 0.2, 0.3))
    st = oracle.render(sc, cam, cfg)
    ib, Tb = brute.render_lin(sc, cam, cfg)
    np.testing.assert_allclose(st["fwd"]["img"], ib, atol=1e-13)
    np.testing.assert_allclose(st["fwd"]["Tfinal"], Tb, atol=1e-13)
    assert (st["fwd"]["nblend"] > 0).mean() > 0.03


def test_footprint_lies_in_the_rect():
    sc = scene_clusters(200, seed=4, n_clusters=3, box=1.0, lo=0.01, hi=0.3)
    cam = camera_look_at((0.1, 0.2, -3.8), 100, 80)
    pr = oracle.project(sc, cam, _cfg())
    ys, xs = np.mgrid[0:cam.height, 0:cam.width]
    pxy = np.stack([xs.ravel(), ys.ravel()], 1)
    n = 0
    for i in np.nonzero(pr["tc"] > 0)[0][:80]:
        ch = oracle.lin_chord(np.repeat(pr["rec"][i][None], len(pxy), 0), pxy)
        hit = ch > 0
        x0, y0, x1, y1 = pr["rect"][i]
        tx, ty = pxy[hit, 0] // 16, pxy[hit, 1] // 16
        assert np.all((tx >= x0) & (tx < x1) & (ty >= y0) & (ty < y1))
        n += hit.sum()
    assert n > 300
