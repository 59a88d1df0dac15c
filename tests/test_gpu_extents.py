"""Parity of the opacity-aware extents (compute_extents of the listing
"Implementation of XPR-3DGS" with the opacity) on the HIP path: projection
rects and tile counts bit-exact with the FP64 oracle outside the guard band,
binning bit-exact, compositing within 1e-5 and gradients within 1e-3, the
image independent of the tile size at any opacity, and the combination with
the per-(Gaussian, tile) cull."""
import functools

import numpy as np
import pytest

import oracle
from gpu_util import (cam32, check_binning, check_binning_cull, check_forward, check_projection,
                      guard_records, log, ocfg_of, rec9, rel_check, run_gpu)
from paper_2606_11529_amd import renderer as R
from synth import camera_front, camera_look_at, random_cameras, scene_clusters, scene_uniform_cube

pytestmark = pytest.mark.gpu


def _case(name):
    if name == "cube_10k_256":
        return scene_uniform_cube(10_000, 0), camera_front(256, 256), R.Config(sh_degree=0)
    if name == "ragged_t8":
        sc = scene_clusters(3000, seed=5, n_clusters=6, box=1.2, lo=0.005, hi=0.4)
        return sc, camera_look_at((0.7, -0.4, -3.2), 77, 45), R.Config(tile=8, sh_degree=3)
    if name == "clusters_1M_1297x840":
        sc = scene_clusters(1_000_000, seed=0)
        return sc, random_cameras(1, 0, (1297, 840))[0], R.Config(sh_degree=3)
    raise KeyError(name)


CASES = ["cube_10k_256", "ragged_t8", "clusters_1M_1297x840"]


@functools.lru_cache(maxsize=3)
def _run(name):
    sc, cam, cfg = _case(name)
    cfg.opacity_extents = True
    rng = np.random.default_rng(1)
    dimg = rng.normal(size=(3, cam.height, cam.width)).astype(np.float32) / (3 * cam.width * cam.height)
    log(f"[gpu extents] case={name} n={sc.n} {cam.width}x{cam.height} tile={cfg.tile}")
    return sc, cam, cfg, dimg, run_gpu(sc, cam, cfg, dimgs=[dimg])


@pytest.mark.parametrize("name", CASES)
def test_extents_projection_and_binning(name):
    sc, cam, cfg, _, g = _run(name)
    idx = None
    if sc.n > 200_000:
        idx = np.sort(np.random.default_rng(2).choice(sc.n, 200_000, replace=False))
    nguard, n = check_projection(sc, cam, cfg, g, idx=idx)
    tx, ty = oracle.tiles(cam, ocfg_of(cfg))
    check_binning(g, (tx, ty))
    log(f"[E1] {name}: {n} Gaussians, {nguard} guard, I={g['I']} bit-exact")


@pytest.mark.parametrize("name", CASES)
def test_extents_forward_backward(name):
    sc, cam, cfg, dimg, g = _run(name)
    emax, nguard, ref_f = check_forward(g, cam, cfg)
    oc = ocfg_of(cfg)
    g9 = oracle.render_bwd(rec9(g["splat"]), g["vals"], g["ranges"], cam.width, cam.height, oc,
                           dimg.astype(np.float64))
    tx, _ = oracle.tiles(cam, oc)
    excl = guard_records(ref_f, g["ncontrib"][0], g["ranges"], g["vals"], cfg.tile, tx)
    mask = np.ones(sc.n, bool)
    mask[excl] = False
    w2 = rel_check(g["grad2d"], g9, "grad2d", mask)
    ref_p = oracle.project_bwd(sc, cam32(cam), oc, g["grad2d"].astype(np.float64))
    for k in ("means", "scales", "quats", "opacities", "sh"):
        gk, rk = g["grads"][k], ref_p[k]
        gk = gk.reshape(-1, sc.n).T if gk.ndim > 1 else gk
        rk = rk.reshape(-1, sc.n).T if rk.ndim > 1 else rk
        rel_check(gk, rk, k, mask & (g["tc"] > 0))
    log(f"[E2] {name}: max-abs {emax:.2e}, guard pixels {nguard}, grad2d {w2:.2e} x bound")


@pytest.mark.parametrize("opaque", [False, True])
def test_extents_tile_size_invariance(opaque):
    sc = scene_clusters(4000, seed=4, n_clusters=8, box=1.5, lo=0.004, hi=0.3)
    if opaque:
        sc.opacities[:] = np.float32(0.98)
    cam = camera_look_at((0.2, -0.4, -4.0), 100, 75)
    a = run_gpu(sc, cam, R.Config(tile=8, opacity_extents=True))
    b = run_gpu(sc, cam, R.Config(tile=16, opacity_extents=True))
    c = run_gpu(sc, cam, R.Config(tile=32, opacity_extents=True))
    assert np.array_equal(a["image"][0], b["image"][0])
    assert np.array_equal(a["image"][0], c["image"][0])


def test_extents_with_cull():
    sc = scene_clusters(20000, seed=9, n_clusters=8, box=1.5, lo=0.004, hi=0.3)
    cam = camera_look_at((0.3, 0.2, -4.0), 160, 120)
    cfg = R.Config(opacity_extents=True, tile_cull=True)
    g = run_gpu(sc, cam, cfg)
    g0 = run_gpu(sc, cam, R.Config(opacity_extents=True))
    check_binning_cull(g, cam, cfg, oracle.tiles(cam, ocfg_of(cfg)))
    check_forward(g, cam, cfg)
    d = np.abs(g["image"][0] - g0["image"][0]).max()
    assert d <= 1e-5, d
    log(f"[E3] extents+cull: kept {g['I']} of {g0['I']}")
