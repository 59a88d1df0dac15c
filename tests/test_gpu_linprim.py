"""Parity of the LinPrim forward path (listing "Implementation of
XPR-LinPrim") on the HIP path with the FP64 oracle, through the C-ABI: the
projection (floats within rounding bounds, rects and tile counts bit-exact
outside the guard band), binning bit-exact on the Euclidean depth,
compositing within 1e-5 max-abs with n_contrib exact; with tile_cull the
lists equal the oracle's kept pairs (its per-tile chord bound) bit-exactly
outside the guard band and the images stay within the tolerance of the uncut
ones. The backward: the 16 per-record values (u, v, sigma, colour, the rows
of A^-1, a zero) and the parameter gradients within 1e-3 relative of the
oracle's, each stage fed the GPU's previous stage, records a guard-band
decision can reach excluded; the same with tile_cull; accumulate and a
two-scene batch against per-view sums."""
import functools

import numpy as np
import pytest
import torch

import oracle
from gpu_util import (cam32, check_binning, check_binning_cull, guard_records, log, ocfg_of,
                      rel_check, run_gpu, TOL_PIXEL)
from paper_2606_11529_amd import renderer as R
from helpers import axis_camera, hand_scene
from synth import camera_front, camera_look_at, random_cameras, scene_clusters, scene_uniform_cube

pytestmark = pytest.mark.gpu

ULP = 2.0 ** -23


def _case(name):
    if name == "cube_10k_256":
        return scene_uniform_cube(10_000, 0), camera_front(256, 256), R.Config(sh_degree=0)
    if name == "ragged_t8":
        sc = scene_clusters(3000, seed=5, n_clusters=6, box=1.2, lo=0.005, hi=0.4)
        return sc, camera_look_at((0.7, -0.4, -3.2), 77, 45), R.Config(tile=8, sh_degree=3)
    if name == "ragged_t16":
        sc = scene_clusters(3000, seed=6, n_clusters=6, box=1.2, lo=0.005, hi=0.4, sh_degree=1)
        return sc, camera_look_at((-0.3, 0.5, -3.9), 101, 67), R.Config(sh_degree=1)
    if name == "axis_grid_t8":
        # axis-aligned octahedra in front of an axis camera: the ones on the
        # horizontal axis have slab pairs with equal x slopes (a_i == a_j)
        g = np.stack(np.meshgrid(np.linspace(-1, 1, 9), np.linspace(-0.6, 0.6, 7), [4.0]),
                     -1).reshape(-1, 3)
        g[:, 0] += 0.013
        sc = hand_scene(g, [[0.12, 0.09, 0.05]], opac=0.8)
        return sc, axis_camera(150, 97, f=120.0), R.Config(tile=8, sh_degree=0)
    if name == "clusters_1M_1297x840":
        sc = scene_clusters(1_000_000, seed=0)
        return sc, random_cameras(1, 0, (1297, 840))[0], R.Config(sh_degree=3)
    raise KeyError(name)


CASES = ["cube_10k_256", "ragged_t8", "ragged_t16", "axis_grid_t8", "clusters_1M_1297x840"]


def _dimg(cam, seed=1):
    rng = np.random.default_rng(seed)
    return rng.normal(size=(3, cam.height, cam.width)).astype(np.float32) / (
        3 * cam.width * cam.height)


@functools.lru_cache(maxsize=1)
def _run(name, cull=False):
    sc, cam, cfg = _case(name)
    cfg.method = "linprim"
    cfg.tile_cull = cull
    log(f"[gpu linprim] case={name} n={sc.n} {cam.width}x{cam.height} tile={cfg.tile} "
        f"cull={cull}")
    return sc, cam, cfg, run_gpu(sc, cam, cfg, dimgs=[_dimg(cam)])


def _check_projection(sc, cam, cfg, g, idx):
    ref = oracle.project(sc.subset(idx), cam32(cam), ocfg_of(cfg))
    got = g["splat"][idx, :17].astype(np.float64)
    ok = ~ref["guard"].astype(bool)
    assert np.array_equal(g["tc"][idx][ok], ref["tc"][ok]), "tc mismatch"
    vr = ok & (ref["tc"] > 0)
    assert np.array_equal(g["rect"][idx][vr], ref["rect"][vr]), "rect mismatch"
    m = (ref["tc"] > 0) & (g["tc"][idx] > 0)
    rr, gg = ref["rec"][m], got[m]
    for cols, name, k in (((0, 1), "mean2D", 1), ((2,), "sigma", 4), ((6, 7), "extents", 2)):
        c = list(cols)
        scale = np.maximum(1.0, np.abs(rr[:, c]))
        err = (np.abs(gg[:, c] - rr[:, c]) / scale).max(initial=0)
        assert err <= k * ULP, f"{name} error {err}"
    assert np.abs(gg[:, 3:6] - rr[:, 3:6]).max(initial=0) <= 1e-6, "colour"
    c = rr[:, 8:17].reshape(-1, 3, 3)
    rowmax = np.abs(c).max(axis=2, keepdims=True)
    lim = 2 * ULP * np.abs(c) + 1e-10 * rowmax
    worst = (np.abs(gg[:, 8:17].reshape(-1, 3, 3) - c) / lim).max(initial=0)
    assert worst <= 1.0, f"slab rows error {worst} x bound"
    d_err = np.abs(g["depth"][idx][m] - ref["depth"][m]) / np.maximum(1.0, ref["depth"][m])
    assert d_err.max(initial=0) <= ULP
    return int((~ok).sum())


def _check_forward(g, cam, cfg):
    oc = ocfg_of(cfg)
    rec = g["splat"][:, :17].astype(np.float64)
    ref = oracle.render_fwd_lin(rec, g["vals"], g["ranges"], cam.width, cam.height, oc)
    sel = ~ref["guard"].astype(bool)
    emax = float(np.abs(g["image"][0] - ref["img"])[:, sel].max(initial=0))
    assert emax <= TOL_PIXEL, f"pixel max-abs {emax}"
    assert np.array_equal(g["ncontrib"][0][sel], ref["ncontrib"][sel]), "n_contrib differs"
    terr = np.abs(g["Tfinal"][0][sel] - ref["Tfinal"][sel]).max(initial=0)
    assert terr <= TOL_PIXEL, f"T_final {terr}"
    if (~sel).any():
        assert np.abs(g["image"][0] - ref["img"])[:, ~sel].max() <= 1e-2
    return emax, int((~sel).sum())


@pytest.mark.parametrize("name", CASES)
def test_linprim_projection_binning_forward(name):
    sc, cam, cfg, g = _run(name)
    idx = np.arange(sc.n)
    if sc.n > 200_000:
        idx = np.sort(np.random.default_rng(2).choice(sc.n, 200_000, replace=False))
    ng = _check_projection(sc, cam, cfg, g, idx)
    tx, ty = oracle.tiles(cam, ocfg_of(cfg))
    check_binning(g, (tx, ty))
    emax, gp = _check_forward(g, cam, cfg)
    log(f"[L1] {name}: {idx.size} projected ({ng} guard), I={g['I']} bit-exact, "
        f"max-abs {emax:.2e}, guard pixels {gp}, lit {(g['ncontrib'][0] > 0).mean():.3f}")


@pytest.mark.parametrize("name", CASES)
def test_linprim_cull(name):
    _, _, _, g0 = _run(name)
    img0, n0 = g0["image"][0].copy(), g0["I"]
    sc, cam, cfg, g = _run(name, cull=True)
    tx, ty = oracle.tiles(cam, ocfg_of(cfg))
    ref = check_binning_cull(g, cam, cfg, (tx, ty))
    assert ref["I"] == n0 and g["I"] < n0
    emax, gp = _check_forward(g, cam, cfg)
    # culled pairs have alpha < 1/255 at every pixel: the image is the uncut one
    dmax = float(np.abs(g["image"][0] - img0).max())
    assert dmax <= TOL_PIXEL, f"cull changed the image by {dmax}"
    log(f"[L2] {name}: kept {g['I']} of {n0} ({g['I'] / n0:.3f}), guard pairs "
        f"{ref['n_guard']}, max-abs {emax:.2e}, vs uncut {dmax:.1e}")


def _backward_check(sc, cam, cfg, g, dimg, exclude_guard=True):
    """The record gradient against orc_render_bwd_lin on the GPU's records
    and lists, then the parameter gradients against orc_project_bwd_lin fed
    the GPU's record gradient."""
    oc = ocfg_of(cfg)
    rec = g["splat"][:, :17].astype(np.float64)
    ref_f = oracle.render_fwd_lin(rec, g["vals"], g["ranges"], cam.width, cam.height, oc)
    g16 = oracle.render_bwd_lin(rec, g["vals"], g["ranges"], cam.width, cam.height, oc,
                                dimg.astype(np.float64))
    tx, _ = oracle.tiles(cam, oc)
    excl = (guard_records(ref_f, g["ncontrib"][0], g["ranges"], g["vals"], cfg.tile, tx)
            if exclude_guard else np.zeros(0, np.int64))
    mask = np.ones(sc.n, bool)
    mask[excl] = False
    assert g["grad2d"].shape == (sc.n, 16)
    w16 = rel_check(g["grad2d"][:, :15], g16[:, :15], "grad16", mask)
    assert np.all(g["grad2d"][:, 15] == 0)
    listed = np.zeros(sc.n, bool)
    listed[g["vals"]] = True
    assert np.all(g["grad2d"][~listed] == 0), "a record in no list received a gradient"
    ref = oracle.project_bwd_lin(sc, cam32(cam), oc, g["grad2d"].astype(np.float64))
    worst = {}
    m = mask & (g["tc"] > 0)
    for k in ("means", "scales", "quats", "opacities", "sh"):
        gk, rk = g["grads"][k], ref[k]
        gk = gk.reshape(-1, sc.n).T if gk.ndim > 1 else gk
        rk = rk.reshape(-1, sc.n).T if rk.ndim > 1 else rk
        worst[k] = rel_check(gk, rk, k, m)
    return w16, worst, excl.size


@pytest.mark.parametrize("name", CASES)
def test_linprim_backward(name):
    sc, cam, cfg, g = _run(name)
    w16, worst, nex = _backward_check(sc, cam, cfg, g, _dimg(cam))
    lit = (np.abs(g["grad2d"]).sum(axis=1) > 0).sum()
    log(f"[L4] {name}: grad16 {w16:.2e} x bound over {lit} records with a gradient, "
        f"params {worst}, excluded {nex}")


@pytest.mark.parametrize("name", ["ragged_t8", "ragged_t16"])
def test_linprim_backward_with_cull(name):
    """The culled lists give the oracle's gradient on those lists, and (the
    culled pairs blend nowhere) the uncut run's gradient."""
    _, _, _, g0 = _run(name)
    grads0 = {k: v.copy() for k, v in g0["grads"].items()}
    sc, cam, cfg, g = _run(name, cull=True)
    w16, worst, nex = _backward_check(sc, cam, cfg, g, _dimg(cam))
    for k in grads0:
        a, b = g["grads"][k], grads0[k]
        a = a.reshape(-1, sc.n).T if a.ndim > 1 else a
        b = b.reshape(-1, sc.n).T if b.ndim > 1 else b
        rel_check(a, b, f"cut vs uncut {k}")
    log(f"[L5] {name} cull: grad16 {w16:.2e}, params {worst}, excluded {nex}")


def test_linprim_backward_clamped_opacity():
    """An octahedron whose alpha passes alpha_max through its centre (no
    gradient to its sigma or slabs there) and a colour channel clamped to 0
    (none to its SH coefficients), beside ordinary octahedra."""
    sh = np.zeros((4, 16, 3))
    sh[:, 0, :] = [[1.2, 0.3, 0.6], [0.4, -2.5, 0.8], [0.9, 0.9, 0.1], [0.2, 0.5, 1.1]]
    rng = np.random.default_rng(11)
    sh[:, 1:, :] = rng.normal(0, 0.05, size=(4, 15, 3))
    means = [[0.05, -0.03, 3.0], [0.15, 0.1, 3.5], [-0.3, 0.2, 4.0], [0.02, 0.03, 2.5]]
    scales = [[0.15, 0.1, 0.12], [0.2, 0.15, 0.18], [0.3, 0.2, 0.25], [0.25, 0.3, 0.8]]
    quats = rng.normal(size=(4, 4)) * [1, 0.2, 0.2, 0.2]
    quats[3] = [1.0, 0.02, -0.03, 0.01]
    sc = hand_scene(means, scales, quats=quats, opac=[0.7, 0.6, 0.5, 0.95], sh_degree=3, sh=sh)
    cam = axis_camera(88, 72, f=80.0)
    cfg = R.Config(method="linprim", sh_degree=3, tile=8, bg=(0.2, 0.1, 0.05))
    dimg = _dimg(cam, seed=5)
    g = run_gpu(sc, cam, cfg, dimgs=[dimg])
    rec = g["splat"][:, :17].astype(np.float64)
    assert (g["tc"] > 0).all() and rec[1, 4] == 0.0
    px = np.array([[x, y] for y in range(cam.height) for x in range(cam.width)], np.int32)
    ch = oracle.lin_chord(np.repeat(rec[3:4], len(px), 0), px)
    assert (-np.expm1(-rec[3, 2] * ch)).max() > 0.99, "the long octahedron must clamp"
    w16, worst, nex = _backward_check(sc, cam, cfg, g, dimg)
    assert np.all(g["grads"]["sh"].reshape(16, 3, 4)[:, 1, 1] == 0), "clamped green passed"
    log(f"[L6] clamp scene: grad16 {w16:.2e}, params {worst}, excluded {nex}")


def test_linprim_backward_accumulate_and_batch():
    """accumulate adds to the buffers; a batch of three views over two
    scenes gives each scene the sum of its views' gradients from one call
    (within the gradient tolerance: the float atomics sum in another
    order)."""
    sa = scene_clusters(3000, seed=11, n_clusters=4, box=1.2, lo=0.01, hi=0.25, sh_degree=1)
    sb = scene_clusters(2000, seed=12, n_clusters=3, box=1.0, lo=0.01, hi=0.3, sh_degree=1)
    cams = [camera_look_at((0.3, -0.2, -3.9), 90, 70), camera_look_at((-0.4, 0.1, -4.1), 64, 80),
            camera_look_at((0.1, 0.4, -3.7), 72, 60)]
    cfg = R.Config(method="linprim", sh_degree=1)
    scenes = [R.Scene.from_host(sa), R.Scene.from_host(sb)]
    vs = [0, 1, 0]
    views = R.Views(scenes, cams, vs, cfg)
    proj = R.xpr_project(views, cfg)
    bins = R.xpr_bin_sort(views, cfg, proj)
    frame = R.xpr_render_fwd(views, cfg, proj, bins)
    dimgs = [_dimg(c, seed=20 + i) for i, c in enumerate(cams)]
    flat = torch.cat([torch.from_numpy(d).reshape(-1) for d in dimgs]).cuda()
    grads, _ = R.xpr_render_bwd(views, cfg, proj, bins, frame, flat)
    per = [None, None]
    for v, (cam, s) in enumerate(zip(cams, vs)):
        one = run_gpu([sa, sb][s], cam, cfg, dimgs=[dimgs[v]])
        if per[s] is None:
            per[s] = {k: x.astype(np.float64) for k, x in one["grads"].items()}
        else:
            for k in per[s]:
                per[s][k] += one["grads"][k]
    for s in range(2):
        n = scenes[s].n
        for k in per[s]:
            got = grads[s][k].cpu().numpy().astype(np.float64)
            got = got.reshape(-1, n).T if got.ndim > 1 else got
            ref = per[s][k].reshape(-1, n).T if per[s][k].ndim > 1 else per[s][k]
            rel_check(got, ref, f"scene {s} {k}")
    acc = [{k: t.clone() for k, t in gs.items()} for gs in grads]
    R.xpr_render_bwd(views, cfg, proj, bins, frame, flat, grads=acc, accumulate=True)
    for s in range(2):
        for k in acc[s]:
            rel_check((acc[s][k] - grads[s][k]).cpu().numpy(), grads[s][k].cpu().numpy(),
                      f"accumulate {s} {k}")
    log(f"[L7] batch of 3 views over 2 scenes, {views.records} records, I={bins.count}")


def test_linprim_cull_empty_and_everything_culled():
    from synth import scene_uniform_cube
    cam = camera_look_at((0, 0, -4.0), 64, 48)
    g = run_gpu(scene_uniform_cube(10, 0).subset(np.arange(0)), cam,
                R.Config(method="linprim", tile_cull=True, sh_degree=0))
    assert g["I"] == 0
    # a density this low keeps sigma * chord below -log(1 - 1/255) everywhere
    sc = scene_uniform_cube(300, 2)
    sc.opacities[:] = np.float32(1e-4)
    cfg = R.Config(method="linprim", tile_cull=True, sh_degree=0)
    g = run_gpu(sc, cam, cfg)
    g0 = run_gpu(sc, cam, R.Config(method="linprim", sh_degree=0))
    assert g0["I"] > 0 and g["I"] == 0
    check_binning_cull(g, cam, cfg, oracle.tiles(cam, ocfg_of(cfg)))
    assert np.array_equal(g["image"][0], g0["image"][0])


@pytest.mark.parametrize("tile", [8, 16, 32])
def test_linprim_cull_tile_sizes(tile):
    sc = scene_clusters(2500, seed=9, n_clusters=5, box=1.2, lo=0.004, hi=0.35)
    cam = camera_look_at((0.6, 0.3, -3.6), 149, 93)
    cfg = R.Config(method="linprim", tile_cull=True, tile=tile, sh_degree=1)
    g = run_gpu(sc, cam, cfg)
    g0 = run_gpu(sc, cam, R.Config(method="linprim", tile=tile, sh_degree=1))
    ref = check_binning_cull(g, cam, cfg, oracle.tiles(cam, ocfg_of(cfg)))
    assert ref["I"] == g0["I"] and g["I"] < g0["I"]
    _check_forward(g, cam, cfg)
    assert float(np.abs(g["image"][0] - g0["image"][0]).max()) <= TOL_PIXEL
    log(f"[L3] tile {tile}: kept {g['I']} of {g0['I']}")


def test_linprim_cull_batched_views_equal_single_views():
    sc = scene_clusters(4000, seed=10, n_clusters=6, box=1.2, lo=0.004, hi=0.3)
    cams = random_cameras(3, 4, [(64, 48), (97, 61), (128, 96)], radius=4.5)
    cfg = R.Config(method="linprim", tile_cull=True, sh_degree=1)
    batch = run_gpu(sc, cams, cfg)
    for v, cam in enumerate(cams):
        one = run_gpu(sc, cam, cfg)
        assert np.array_equal(batch["image"][v], one["image"][0]), v
        assert np.array_equal(batch["ncontrib"][v], one["ncontrib"][0]), v
