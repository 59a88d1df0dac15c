"""Pins of the oracle's LinPrim tile_cull (Listing "Implementation of
XPR-LinPrim", tile_cull; the per-tile upper bound and the cull predicate of
the XPR-LinPrim section): the bound of an axis-aligned on-axis octahedron in
closed form (there it equals the longest chord over the tile box), the bound
of general octahedra against one linear program per ordered slab pair, the
bound above every pixel's chord and below twice the smallest slab
half-width, and the rendered image unchanged by the cull (a culled pair has
alpha below the gate at every pixel of its tile); slabs parallel to the
viewing rays drop out of the bound."""
import math

import numpy as np
import pytest
from scipy.optimize import linprog

import oracle
from helpers import axis_camera, hand_scene
from synth import Camera, camera_look_at, scene_clusters


def _cfg(**kw):
    kw.setdefault("sh_degree", 0)
    kw.setdefault("method", "linprim")
    return oracle.OracleConfig(**kw)


def _box(tx, ty, W, H, t):
    """Pixel-sample box of a tile: first and last pixel index in x and y."""
    return tx * t, min(tx * t + t - 1, W - 1), ty * t, min(ty * t + t - 1, H - 1)


def _bounds(rec, pairs, W, H, cfg):
    """Chord bound (power / sigma) and the cull outputs of (record, tile) pairs."""
    idx = np.array([p[0] for p in pairs])
    txy = np.array([p[1] for p in pairs], np.int32)
    keep, power, level, guard = oracle.tile_cull(rec[idx], txy, W, H, cfg)
    return power / rec[idx, 2], keep, level, guard


@pytest.mark.parametrize("centre", ["inside", "beyond_border"])
def test_on_axis_octahedron_bound_closed_form(centre):
    # A = diag(f sx / z, f sy / z, sz): the octahedron is
    # |dx| / a + |dy| / b + |tau| / sz <= 1 and the bound over a box equals
    # the longest chord in it, 2 sz (1 - dxn / a - dyn / b) (>= 0), with dxn,
    # dyn the distances from mu_2D to the box (clipped to the image: with
    # the centre beyond the border, the last tiles' boxes end at W - 1, H - 1)
    W, H, f, z0 = 97, 75, 110.0, 4.0
    sx, sy, sz = 0.35, 0.25, 0.1
    cam = axis_camera(W, H, f=f)
    if centre == "beyond_border":
        cam = Camera(R=cam.R, t=cam.t, fx=f, fy=f, cx=W + 2.5, cy=H + 1.5, width=W, height=H)
    sc = hand_scene([[0, 0, z0]], [[sx, sy, sz]], opac=0.6)
    for t in (8, 16):
        cfg = _cfg(tile_w=t, tile_h=t)
        pr = oracle.project(sc, cam, cfg)
        r = pr["rec"]
        u, v = r[0, 0], r[0, 1]
        a, b = f * float(np.float32(sx)) / z0, f * float(np.float32(sy)) / z0
        s = float(np.float32(sz))
        txs, tys = (W + t - 1) // t, (H + t - 1) // t
        pairs = [(0, (x, y)) for y in range(tys) for x in range(txs)]
        bound, keep, level, _ = _bounds(r, pairs, W, H, cfg)
        n_zero = 0
        for k, (_, (x, y)) in enumerate(pairs):
            X0, X1, Y0, Y1 = _box(x, y, W, H, t)
            dxn = max(X0 - u, u - X1, 0.0)
            dyn = max(Y0 - v, v - Y1, 0.0)
            want = max(0.0, 2 * s * (1 - dxn / a - dyn / b))
            assert bound[k] == pytest.approx(want, rel=1e-12, abs=1e-14), (t, x, y)
            assert keep[k] == (r[0, 2] * bound[k] >= level[k])
            n_zero += want == 0.0
        assert level[0] == pytest.approx(-math.log1p(-cfg.alpha_min), rel=1e-12)
        assert 0 < n_zero < len(pairs)


def _pair_lp(c, X0, X1, Y0, Y1, u, v, i, j):
    """max over the box of s_i^hi - s_j^lo, as a linear program in (x, y)."""
    def slab(k):
        e1 = -1.0 if k & 2 else 1.0
        e2 = -1.0 if k & 1 else 1.0
        return c[0] + e1 * c[1] + e2 * c[2]
    ni, nj = slab(i), slab(j)
    # s_i^hi - s_j^lo = h_i + h_j + (a_i - a_j) (x - u) + (b_i - b_j) (y - v)
    ai, bi, hi_ = -ni[0] / ni[2], -ni[1] / ni[2], 1 / abs(ni[2])
    aj, bj, hj = -nj[0] / nj[2], -nj[1] / nj[2], 1 / abs(nj[2])
    res = linprog([-(ai - aj), -(bi - bj)], bounds=[(X0, X1), (Y0, Y1)], method="highs")
    x, y = res.x
    return hi_ + hj + (ai - aj) * (x - u) + (bi - bj) * (y - v)


def test_bound_matches_pairwise_linear_programs():
    sc = scene_clusters(60, seed=5, n_clusters=2, box=0.8, lo=0.02, hi=0.25)
    cam = camera_look_at((0.3, -0.2, -3.6), 90, 70)
    cfg = _cfg(tile_w=8, tile_h=8)
    pr = oracle.project(sc, cam, cfg)
    rec = pr["rec"]
    rng = np.random.default_rng(5)
    pairs = []
    for i in np.nonzero(pr["tc"] > 0)[0]:
        x0, y0, x1, y1 = pr["rect"][i]
        for _ in range(4):
            pairs.append((i, (int(rng.integers(x0, x1)), int(rng.integers(y0, y1)))))
    bound, _, _, _ = _bounds(rec, pairs, cam.width, cam.height, cfg)
    for k, (i, (x, y)) in enumerate(pairs):
        c = rec[i, 8:17].reshape(3, 3)
        X0, X1, Y0, Y1 = _box(x, y, cam.width, cam.height, 8)
        g = [_pair_lp(c, X0, X1, Y0, Y1, rec[i, 0], rec[i, 1], a, b)
             for a in range(4) for b in range(4)]
        want = max(0.0, min(g))
        assert bound[k] == pytest.approx(want, rel=1e-9, abs=1e-12 * max(g)), (i, x, y)
    assert len(pairs) > 150
    assert (bound > 0).mean() > 0.3


def test_bound_covers_every_pixel_chord():
    sc = scene_clusters(80, seed=6, n_clusters=3, box=1.0, lo=0.01, hi=0.3)
    cam = camera_look_at((0.1, 0.2, -3.8), 72, 56)
    t = 8
    cfg = _cfg(tile_w=t, tile_h=t)
    pr = oracle.project(sc, cam, cfg)
    rec = pr["rec"]
    pairs = []
    for i in np.nonzero(pr["tc"] > 0)[0]:
        x0, y0, x1, y1 = pr["rect"][i]
        pairs += [(i, (x, y)) for y in range(y0, y1) for x in range(x0, x1)]
    bound, keep, level, _ = _bounds(rec, pairs, cam.width, cam.height, cfg)
    n_culled = n_tight = 0
    for k, (i, (x, y)) in enumerate(pairs):
        X0, X1, Y0, Y1 = _box(x, y, cam.width, cam.height, t)
        ys, xs = np.mgrid[Y0:Y1 + 1, X0:X1 + 1]
        pxy = np.stack([xs.ravel(), ys.ravel()], 1)
        ch = oracle.lin_chord(np.repeat(rec[i][None], len(pxy), 0), pxy)
        top = max(ch.max(), 0.0)
        c = rec[i, 8:17].reshape(3, 3)
        nz = np.array([c[0, 2] + e1 * c[1, 2] + e2 * c[2, 2]
                       for e1 in (1, -1) for e2 in (1, -1)])
        assert top <= bound[k] * (1 + 1e-12) + 1e-15
        assert bound[k] <= 2 / np.abs(nz).max() * (1 + 1e-15)
        if not keep[k]:
            n_culled += 1
            # every pixel's alpha is below the gate
            assert np.all(-np.expm1(-rec[i, 2] * np.maximum(ch, 0)) < cfg.alpha_min)
        n_tight += top > 0.5 * bound[k]
    assert n_culled > 0.1 * len(pairs)
    assert n_tight > 0.3 * len(pairs)


@pytest.mark.parametrize("seed,tile", [(0, 16), (3, 8)])
def test_cull_leaves_the_image_unchanged(seed, tile):
    sc = scene_clusters(200, seed=seed, n_clusters=3, box=1.0, lo=0.01, hi=0.25)
    cam = camera_look_at((0.5, -0.3, -4.5), 128, 96)
    base = dict(sh_degree=3, tile_w=tile, tile_h=tile, bg=(0.1, 0.2, 0.3))
    a = oracle.render(sc, cam, _cfg(**base))
    b = oracle.render(sc, cam, _cfg(tile_cull=True, **base))
    assert b["bins"]["I"] == a["bins"]["I"]
    assert b["bins"]["I_kept"] < 0.92 * a["bins"]["I"]
    for key in ("img", "Tfinal", "nblend"):
        assert np.array_equal(a["fwd"][key], b["fwd"][key]), key
    assert (a["fwd"]["nblend"] > 0).mean() > 0.03


def test_flat_slabs_drop_out_of_the_bound():
    # rows c0 = (1/a, 0, 1/s), c1 = (0, 1/b, 0), c2 = (0, 0, 1/s): slabs
    # c0 +- c1 - c2 have n_z = 0 (they bound only |dx / a +- dy / b| <= 1);
    # the other two give the chord s (1 - |dy| / b), so the bound over a box
    # is max(0, s (1 - dyn / b))
    W, H, t = 64, 48, 8
    a, b, s = 9.0, 6.0, 0.2
    u, v = 30.3, 21.6
    rec = np.zeros(17)
    rec[:3] = u, v, 5.0
    rec[8:17] = [1 / a, 0, 1 / s, 0, 1 / b, 0, 0, 0, 1 / s]
    cfg = _cfg(tile_w=t, tile_h=t)
    pairs = [(0, (x, y)) for y in range(H // t) for x in range(W // t)]
    bound, _, _, _ = _bounds(rec[None], pairs, W, H, cfg)
    ys, xs = np.mgrid[0:H, 0:W]
    ch = oracle.lin_chord(np.repeat(rec[None], W * H, 0),
                          np.stack([xs.ravel(), ys.ravel()], 1)).reshape(H, W)
    for k, (_, (x, y)) in enumerate(pairs):
        X0, X1, Y0, Y1 = _box(x, y, W, H, t)
        dyn = max(Y0 - v, v - Y1, 0.0)
        assert bound[k] == pytest.approx(max(0.0, s * (1 - dyn / b)), rel=1e-12, abs=1e-15)
        assert ch[Y0:Y1 + 1, X0:X1 + 1].max() <= bound[k] * (1 + 1e-12) + 1e-15
    # the flat slabs still cut the footprint to the diamond |dx/a| + |dy/b| <= 1
    dx, dy = xs - u, ys - v
    assert np.all(ch[np.abs(dx) / a + np.abs(dy) / b > 1 + 1e-9] <= 0)
    assert (ch > 0).sum() > 50
