"""Parity of the 3DGUT forward path (listing "Implementation of XPR-3DGUT")
on the HIP path with the FP64 oracle, through the C-ABI: the UT projection
(floats within rounding bounds, rects and tile counts bit-exact outside the
guard band), binning bit-exact (also with the extended-bound tile cull),
compositing within 1e-5 max-abs with n_contrib exact, the image independent
of the sort strategy, and the backward entry points refusing the method."""
import functools

import numpy as np
import pytest

import oracle
from gpu_util import (cam32, check_binning, check_binning_cull, log, ocfg_of, run_gpu,
                      TOL_PIXEL)
from paper_2606_11529_amd import _lib as L
from paper_2606_11529_amd import renderer as R
from synth import camera_front, camera_look_at, random_cameras, scene_clusters, scene_uniform_cube

pytestmark = pytest.mark.gpu

ULP = 2.0 ** -23


def _case(name):
    if name == "cube_10k_256":
        return scene_uniform_cube(10_000, 0), camera_front(256, 256), R.Config(sh_degree=0)
    if name == "ragged_t8":
        sc = scene_clusters(3000, seed=5, n_clusters=6, box=1.2, lo=0.005, hi=0.4)
        return sc, camera_look_at((0.7, -0.4, -3.2), 77, 45), R.Config(tile=8, sh_degree=3)
    if name == "ragged_t16_ext":
        sc = scene_clusters(3000, seed=6, n_clusters=6, box=1.2, lo=0.005, hi=0.4, sh_degree=1)
        return (sc, camera_look_at((-0.3, 0.5, -3.9), 101, 67),
                R.Config(sh_degree=1, opacity_extents=True))
    if name == "ragged_t32":
        sc = scene_clusters(4000, seed=7, n_clusters=6, box=1.2, lo=0.005, hi=0.4, sh_degree=2)
        return sc, camera_look_at((0.4, 0.3, -4.0), 150, 97), R.Config(tile=32, sh_degree=2)
    if name == "clusters_1M_1297x840":
        sc = scene_clusters(1_000_000, seed=0)
        return sc, random_cameras(1, 0, (1297, 840))[0], R.Config(sh_degree=3)
    raise KeyError(name)


CASES = ["cube_10k_256", "ragged_t8", "ragged_t16_ext", "ragged_t32", "clusters_1M_1297x840"]


@functools.lru_cache(maxsize=2)
def _run(name, cull=False):
    sc, cam, cfg = _case(name)
    cfg.method = "3dgut"
    cfg.tile_cull = cull
    log(f"[gpu gut] case={name} cull={cull} n={sc.n} {cam.width}x{cam.height} tile={cfg.tile}")
    return sc, cam, cfg, run_gpu(sc, cam, cfg)


def _check_projection(sc, cam, cfg, g, idx):
    sub = sc.subset(idx)
    ref = oracle.project(sub, cam32(cam), ocfg_of(cfg))
    got = g["splat"][idx, :21].astype(np.float64)
    guard = ref["guard"].astype(bool)
    ok = ~guard
    assert np.array_equal(g["tc"][idx][ok], ref["tc"][ok]), "tc mismatch"
    vr = ok & (ref["tc"] > 0)
    assert np.array_equal(g["rect"][idx][vr], ref["rect"][vr]), "rect mismatch"
    m = (ref["tc"] > 0) & (g["tc"][idx] > 0)
    rr = ref["rec"][m]
    gg = got[m]
    # FP64 on both sides from the same float32 inputs, rounded to float32
    for cols, name in (((0, 1), "mean2D"), ((9, 10, 11), "ro"), (tuple(range(12, 21)), "M")):
        c = list(cols)
        scale = np.maximum(1.0, np.abs(rr[:, c]).max(axis=1, keepdims=True))
        err = (np.abs(gg[:, c] - rr[:, c]) / scale).max(initial=0)
        assert err <= 2 * ULP, f"{name} error {err}"
    d_err = np.abs(g["depth"][idx][m] - ref["depth"][m]) / np.maximum(1.0, np.abs(ref["depth"][m]))
    assert d_err.max(initial=0) <= ULP
    assert np.abs(gg[:, 6:9] - rr[:, 6:9]).max(initial=0) <= 1e-6, "colour"
    o_err = np.abs(gg[:, 5] - rr[:, 5]) / np.maximum(rr[:, 5], 1e-30)
    assert o_err.max(initial=0) <= 4 * ULP, f"o' error {o_err.max()}"
    cov = ref["cov"][m]
    tr = cov[:, 0] + cov[:, 2]
    det = cov[:, 0] * cov[:, 2] - cov[:, 1] ** 2
    disc = np.sqrt(np.maximum(0, 0.25 * tr * tr - det))
    cond = (0.5 * tr + disc) / np.maximum(0.5 * tr - disc, 1e-300)
    con = rr[:, 2:5]
    scale = np.abs(con).max(axis=1, keepdims=True)
    lim = ULP * np.abs(con) + 2.0 ** -40 * (cond[:, None] + 1.0) * scale
    worst = (np.abs(gg[:, 2:5] - con) / lim).max(initial=0)
    assert worst <= 1.0, f"conic error {worst} x bound"
    return int(guard.sum())


def _check_forward(g, cam, cfg):
    oc = ocfg_of(cfg)
    rec = g["splat"][:, :21].astype(np.float64)
    ref = oracle.render_fwd_gut(rec, g["vals"], g["ranges"], cam32(cam), oc)
    guard = ref["guard"].astype(bool)
    sel = ~guard
    err = np.abs(g["image"][0] - ref["img"])[:, sel]
    emax = float(err.max(initial=0))
    assert emax <= TOL_PIXEL, f"pixel max-abs {emax}"
    assert np.array_equal(g["ncontrib"][0][sel], ref["ncontrib"][sel]), "n_contrib differs"
    terr = np.abs(g["Tfinal"][0][sel] - ref["Tfinal"][sel]).max(initial=0)
    assert terr <= TOL_PIXEL, f"T_final {terr}"
    if guard.any():
        assert np.abs(g["image"][0] - ref["img"])[:, guard].max() <= 1e-2
    return emax, int(guard.sum())


@pytest.mark.parametrize("name", CASES)
def test_gut_projection(name):
    sc, cam, cfg, g = _run(name)
    idx = np.arange(sc.n)
    if sc.n > 200_000:
        idx = np.sort(np.random.default_rng(2).choice(sc.n, 200_000, replace=False))
    ng = _check_projection(sc, cam, cfg, g, idx)
    log(f"[G1] {name}: {idx.size} checked, {ng} guard, visible {(g['tc'] > 0).sum()}")


@pytest.mark.parametrize("name", CASES)
def test_gut_binning_and_forward(name):
    sc, cam, cfg, g = _run(name)
    tx, ty = oracle.tiles(cam, ocfg_of(cfg))
    check_binning(g, (tx, ty))
    emax, ng = _check_forward(g, cam, cfg)
    log(f"[G2] {name}: I={g['I']} bit-exact, max-abs {emax:.2e}, guard pixels {ng}")


@pytest.mark.parametrize("name", ["ragged_t8", "ragged_t16_ext", "ragged_t32", "cube_10k_256"])
def test_gut_with_cull(name):
    sc, cam, cfg, g = _run(name, cull=True)
    tx, ty = oracle.tiles(cam, ocfg_of(cfg))
    check_binning_cull(g, cam, cfg, (tx, ty))
    emax, ng = _check_forward(g, cam, cfg)
    log(f"[G3] {name}: kept {g['I']}, max-abs {emax:.2e}")


def test_gut_sort_modes_agree():
    sc = scene_clusters(4000, seed=3, n_clusters=8, box=1.5, lo=0.004, hi=0.3)
    cam = camera_look_at((0.5, 0.5, -4.5), 120, 90)
    ref = None
    for mode in ("presort", "full", "bands"):
        g = run_gpu(sc, cam, R.Config(method="3dgut", sort_mode=mode))
        if ref is None:
            ref = g
            continue
        assert np.array_equal(g["vals"], ref["vals"]) and np.array_equal(g["image"][0], ref["image"][0])


def test_gut_backward_is_refused():
    sc = scene_clusters(500, seed=4, n_clusters=2, box=1.0, lo=0.01, hi=0.2)
    cam = camera_look_at((0.1, 0.2, -4.0), 48, 32)
    cfg = R.Config(method="3dgut")
    scene = R.Scene.from_host(sc)
    views = R.Views([scene], [cam], [0], cfg)
    proj = R.xpr_project(views, cfg)
    assert proj.splat.shape[1] == 24
    bins = R.xpr_bin_sort(views, cfg, proj)
    frame = R.xpr_render_fwd(views, cfg, proj, bins)
    import torch
    dimg = torch.zeros(3 * views.pixels, dtype=torch.float32, device="cuda")
    with pytest.raises(L.XprError) as e:
        R.xpr_render_bwd(views, cfg, proj, bins, frame, dimg)
    assert e.value.status == L.XPR_ERR_UNSUPPORTED
