"""Pins of the oracle's tile_cull (Listing "Implementation of XPR-3DGS",
function tile_cull, and the XPR-3DGS section's statement of the test): the
smallest power 0.5 (x - mu)^T conic (x - mu) over a tile's pixel box, checked
against closed forms (isotropic: squared distance to a box; axis-aligned:
separable clamps), against a bounded least-squares solver of scipy for a
general conic, against a dense sample of the box from below; and the
invariants that a culled pair has alpha < alpha_min at every pixel of its
tile and that culling leaves the composited image unchanged."""
import math

import numpy as np
import pytest
from scipy.optimize import lsq_linear

import oracle
import oracle.brute as brute
from synth import camera_look_at, scene_clusters

A_MIN = 1.0 / 255.0


def _cfg(**kw):
    kw.setdefault("sh_degree", 0)
    return oracle.OracleConfig(**kw)


def _box(tx, ty, W, H, t=16):
    """Pixel-sample box of tile (tx, ty), clipped to the image."""
    return (tx * t, min(tx * t + t - 1, W - 1), ty * t, min(ty * t + t - 1, H - 1))


def _rec(u, v, a, b, c, o):
    """Shader data (u, v, -0.5 con00, -con01, -0.5 con11, o, colour)."""
    return [u, v, -0.5 * a, -b, -0.5 * c, o, 0.5, 0.5, 0.5]


def _random_pairs(rng, m, W=200, H=150, iso=False, axis=False):
    recs, txy = [], []
    for _ in range(m):
        u, v = rng.uniform(-40, W + 40), rng.uniform(-40, H + 40)
        if iso:
            a = c = math.exp(rng.uniform(math.log(1e-3), math.log(2.0)))
            b = 0.0
        else:
            l1, l2 = np.exp(rng.uniform(math.log(1e-3), math.log(2.0), 2))
            th = rng.uniform(0, math.pi)
            R = np.array([[math.cos(th), -math.sin(th)], [math.sin(th), math.cos(th)]])
            Q = R @ np.diag([l1, l2]) @ R.T
            a, b, c = Q[0, 0], Q[0, 1], Q[1, 1]
            if axis:
                b = 0.0
        o = rng.uniform(A_MIN, 1.0)
        recs.append(_rec(u, v, a, b, c, o))
        txy.append((rng.integers(0, (W + 15) // 16), rng.integers(0, (H + 15) // 16)))
    return np.array(recs), np.array(txy, np.int32), W, H


def test_isotropic_is_squared_distance_to_box():
    rng = np.random.default_rng(0)
    rec, txy, W, H = _random_pairs(rng, 400, iso=True)
    keep, power, level, guard = oracle.tile_cull(rec, txy, W, H, _cfg())
    for k in range(len(rec)):
        u, v, a = rec[k, 0], rec[k, 1], -2 * rec[k, 2]
        x0, x1, y0, y1 = _box(*txy[k], W, H)
        d2 = max(x0 - u, 0, u - x1) ** 2 + max(y0 - v, 0, v - y1) ** 2
        assert power[k] == pytest.approx(0.5 * a * d2, rel=1e-12, abs=1e-300)
        assert level[k] == pytest.approx(math.log(rec[k, 5] / A_MIN), rel=1e-15)
        if not guard[k]:
            assert keep[k] == (0.5 * a * d2 <= level[k])
    assert keep.any() and not keep.all()


def test_axis_aligned_is_separable():
    rng = np.random.default_rng(1)
    rec, txy, W, H = _random_pairs(rng, 400, axis=True)
    _, power, _, _ = oracle.tile_cull(rec, txy, W, H, _cfg())
    for k in range(len(rec)):
        u, v, a, c = rec[k, 0], rec[k, 1], -2 * rec[k, 2], -2 * rec[k, 4]
        x0, x1, y0, y1 = _box(*txy[k], W, H)
        dx = u - min(max(u, x0), x1)
        dy = v - min(max(v, y0), y1)
        assert power[k] == pytest.approx(0.5 * (a * dx * dx + c * dy * dy), rel=1e-12, abs=1e-300)


def test_general_conic_matches_bounded_least_squares_and_dense_sampling():
    # q(x) = |L^T (x - mu)|^2 with conic = L L^T: the smallest q over the
    # box is a bounded-variable least-squares problem (scipy's BVLS solver).
    rng = np.random.default_rng(2)
    rec, txy, W, H = _random_pairs(rng, 300)
    _, power, _, _ = oracle.tile_cull(rec, txy, W, H, _cfg())
    g = np.linspace(0.0, 1.0, 61)
    for k in range(len(rec)):
        u, v = rec[k, 0], rec[k, 1]
        a, b, c = -2 * rec[k, 2], -rec[k, 3], -2 * rec[k, 4]
        Q = np.array([[a, b], [b, c]])
        Lc = np.linalg.cholesky(Q)
        x0, x1, y0, y1 = _box(*txy[k], W, H)
        mu = np.array([u, v])
        res = lsq_linear(Lc.T, Lc.T @ mu, bounds=([x0, y0], [x1, y1]), method="bvls",
                         tol=1e-14)
        d = res.x - mu
        p_ls = 0.5 * float(d @ Q @ d)
        assert power[k] == pytest.approx(p_ls, rel=1e-9, abs=1e-12), k
        # no sample of the box goes below the smallest power
        xs = x0 + (x1 - x0) * g
        ys = y0 + (y1 - y0) * g
        dx, dy = np.meshgrid(xs - u, ys - v)
        p_grid = 0.5 * (a * dx * dx + 2 * b * dx * dy + c * dy * dy)
        assert p_grid.min() >= power[k] * (1 - 1e-12) - 1e-12


def test_not_positive_definite_is_kept():
    rec = np.array([_rec(500.0, 500.0, 1.0, 2.0, 1.0, 0.5), _rec(500.0, 500.0, -1.0, 0.0, 1.0, 0.5)])
    keep, _, _, _ = oracle.tile_cull(rec, np.array([[0, 0], [0, 0]]), 64, 64, _cfg())
    assert keep.all()


def _rect_pairs(pr, tiles_x):
    rows, txy = [], []
    for i in np.nonzero(pr["tc"] > 0)[0]:
        x0, y0, x1, y1 = pr["rect"][i]
        for ty in range(y0, y1):
            for tx in range(x0, x1):
                rows.append(i)
                txy.append((tx, ty))
    return np.array(rows), np.array(txy, np.int32)


@pytest.mark.parametrize("tile", [8, 16])
def test_culled_pairs_reach_no_pixel(tile):
    # every pixel of a culled pair's tile evaluates to alpha < alpha_min
    sc = scene_clusters(1500, seed=3, n_clusters=5, box=1.2, lo=0.004, hi=0.15)
    cam = camera_look_at((0.3, -0.2, -4.0), 96, 72)
    cfg = _cfg(sh_degree=3, tile_w=tile, tile_h=tile)
    pr = oracle.project(sc, cam, cfg)
    tx, _ = oracle.tiles(cam, cfg)
    rows, txy = _rect_pairs(pr, tx)
    keep, _, _, guard = oracle.tile_cull(pr["rec"][rows], txy, cam.width, cam.height, cfg)
    culled = np.nonzero(~keep & ~guard)[0]
    assert culled.size > 0.2 * rows.size
    ys, xs = np.mgrid[0:tile, 0:tile]
    for k in culled:
        r = pr["rec"][rows[k]]
        px = txy[k, 0] * tile + xs
        py = txy[k, 1] * tile + ys
        ok = (px < cam.width) & (py < cam.height)
        dx, dy = px[ok] - r[0], py[ok] - r[1]
        P = r[2] * dx * dx + r[3] * dx * dy + r[4] * dy * dy
        assert (r[5] * np.exp(P)).max() < 1.0 / 255.0


def test_binning_with_cull_is_the_kept_subsequence():
    # the sentinel sort leaves, per tile, the pairs the test keeps in the
    # order of the uncut list; I_kept counts them
    sc = scene_clusters(2000, seed=4, n_clusters=6, box=1.2, lo=0.004, hi=0.2)
    cam = camera_look_at((-0.4, 0.3, -4.2), 111, 70)
    cfg = _cfg(sh_degree=3)
    pr = oracle.project(sc, cam, cfg)
    tx, ty = oracle.tiles(cam, cfg)
    full = oracle.bin_pairs(pr["depth"], pr["rect"], pr["tc"], tx, ty)
    cut = oracle.bin_pairs(pr["depth"], pr["rect"], pr["tc"], tx, ty,
                           (pr["rec"], cam.width, cam.height, cfg))
    assert cut["I"] == full["I"] and cut["n_guard"] == 0
    tid = np.repeat(np.arange(tx * ty), full["ranges"][:, 1] - full["ranges"][:, 0])
    keep, _, _, _ = oracle.tile_cull(pr["rec"][full["vals"]], np.stack([tid % tx, tid // tx], 1),
                                     cam.width, cam.height, cfg)
    assert cut["I_kept"] == int(keep.sum()) < full["I"]
    n = cut["I_kept"]
    assert np.all((cut["keys"][:n] >> np.uint64(32)) < tx * ty)
    assert np.all((cut["keys"][n:] >> np.uint64(32)) == tx * ty)
    s = 0
    for t in range(tx * ty):
        a, b = full["ranges"][t]
        want = full["vals"][a:b][keep[a:b]]
        c0, c1 = cut["ranges"][t]
        got = cut["vals"][c0:c1]
        assert np.array_equal(got, want), t
        if want.size:
            assert c0 == s
        s += want.size
    assert s == n


@pytest.mark.parametrize("seed,tile", [(0, 16), (1, 8)])
def test_cull_leaves_the_image_unchanged(seed, tile):
    # culled pairs only ever carry alpha < alpha_min, which the shader skips
    sc = scene_clusters(1200, seed=seed, n_clusters=4, box=1.0, lo=0.005, hi=0.3)
    cam = camera_look_at((0.4, -0.3, -4.5), 90, 64)
    base = _cfg(sh_degree=3, tile_w=tile, tile_h=tile, bg=(0.1, 0.2, 0.3))
    a = oracle.render(sc, cam, base)
    b = oracle.render(sc, cam, _cfg(sh_degree=3, tile_w=tile, tile_h=tile, bg=(0.1, 0.2, 0.3),
                                   tile_cull=True))
    assert b["bins"]["n_guard"] == 0
    assert b["bins"]["I_kept"] < 0.8 * a["bins"]["I"]
    np.testing.assert_array_equal(a["fwd"]["img"], b["fwd"]["img"])
    # (n_contrib is a list position, which culling shifts; the count blended is not)
    np.testing.assert_array_equal(a["fwd"]["nblend"], b["fwd"]["nblend"])
    np.testing.assert_array_equal(a["fwd"]["Tfinal"], b["fwd"]["Tfinal"])


def test_cull_matches_brute_force_and_gradients_unchanged():
    sc = scene_clusters(150, seed=5, n_clusters=3, box=1.0, lo=0.01, hi=0.3)
    cam = camera_look_at((0.5, -0.3, -4.5), 50, 37)
    cfg = _cfg(sh_degree=3, tile_cull=True)
    st = oracle.render(sc, cam, cfg)
    ib, _ = brute.render(sc, cam, cfg)
    np.testing.assert_allclose(st["fwd"]["img"], ib, atol=1e-13)
    rng = np.random.default_rng(0)
    dimg = rng.normal(size=(3, cam.height, cam.width))
    g_cut = oracle.backward(sc, cam, cfg, dimg, st)
    g_all = oracle.backward(sc, cam, _cfg(sh_degree=3), dimg)
    for k in ("means", "scales", "quats", "opacities", "sh", "grad9"):
        np.testing.assert_allclose(g_cut[k], g_all[k], rtol=1e-12, atol=1e-15)


def test_empty_and_fully_culled():
    e = oracle.bin_pairs(np.zeros(0), np.zeros((0, 4), np.int32), np.zeros(0, np.int32), 3, 2,
                         (np.zeros((0, 9)), 48, 32, _cfg()))
    assert e["I"] == 0 and e["I_kept"] == 0
    # one thin Gaussian far from the corner tiles of its rect: those are culled
    rec = np.array([_rec(24.0, 24.0, 4.0, 0.0, 4.0, 0.9)])
    rect = np.array([[0, 0, 3, 3]], np.int32)
    b = oracle.bin_pairs(np.ones(1), rect, np.array([9], np.int32), 3, 3, (rec, 48, 48, _cfg()))
    assert b["I"] == 9 and b["I_kept"] == 1
    assert tuple(b["ranges"][4]) == (0, 1) and b["ranges"].sum() == 1
