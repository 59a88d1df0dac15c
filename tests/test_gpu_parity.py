"""Stage-wise parity of the HIP path (through the C-ABI) with the FP64 oracle:
P1 projection, P2 binning (bit-exact), P3 forward compositing (1e-5
max-abs), P4 gradients (1e-3 relative), on the small benchmark workload
(10k Gaussians, 256x256, SH degree 0), ragged images with 8x8, 16x16 and
32x32 tiles, and the 1M-Gaussian 1297x840 SH-degree-3 workload."""
import functools

import numpy as np
import pytest

import oracle
from gpu_util import (cam32, check_binning, check_forward, check_projection, guard_records, log,
                      ocfg_of, rec9, rel_check, run_gpu)
from paper_2606_11529_amd import renderer as R
from synth import camera_front, camera_look_at, random_cameras, scene_clusters, scene_uniform_cube

pytestmark = pytest.mark.gpu


def _case(name):
    if name == "cube_10k_256":
        return scene_uniform_cube(10_000, 0), camera_front(256, 256), R.Config(sh_degree=0)
    if name == "ragged_t8":
        sc = scene_clusters(3000, seed=5, n_clusters=6, box=1.2, lo=0.005, hi=0.2)
        return sc, camera_look_at((0.7, -0.4, -4.2), 77, 45), R.Config(tile=8, sh_degree=3)
    if name == "ragged_t16_b64":
        sc = scene_clusters(3000, seed=6, n_clusters=6, box=1.2, lo=0.005, hi=0.2, sh_degree=1)
        return sc, camera_look_at((-0.3, 0.5, -3.9), 101, 67), R.Config(sh_degree=1, lds_batch=64)
    if name == "ragged_t32":
        sc = scene_clusters(4000, seed=7, n_clusters=6, box=1.2, lo=0.005, hi=0.4, sh_degree=2)
        return sc, camera_look_at((0.4, 0.3, -4.0), 150, 97), R.Config(tile=32, sh_degree=2)
    if name == "clusters_1M_1297x840":
        sc = scene_clusters(1_000_000, seed=0)
        cam = random_cameras(1, 0, (1297, 840))[0]
        return sc, cam, R.Config(sh_degree=3)
    raise KeyError(name)


CASES = ["cube_10k_256", "ragged_t8", "ragged_t16_b64", "ragged_t32", "clusters_1M_1297x840"]


@functools.lru_cache(maxsize=2)
def _run(name, sort_mode="presort"):
    sc, cam, cfg = _case(name)
    cfg.sort_mode = sort_mode
    rng = np.random.default_rng(1)
    dimg = rng.normal(size=(3, cam.height, cam.width)).astype(np.float32) / (3 * cam.width * cam.height)
    log(f"[gpu] case={name} sort={sort_mode} n={sc.n} {cam.width}x{cam.height} tile={cfg.tile}")
    g = run_gpu(sc, cam, cfg, dimgs=[dimg])
    return sc, cam, cfg, dimg, g


@pytest.mark.parametrize("name", CASES)
def test_projection(name):
    sc, cam, cfg, _, g = _run(name)
    nguard, n = check_projection(sc, cam, cfg, g)
    log(f"[P1] {name}: {n} Gaussians checked, {nguard} in the guard band")


@pytest.mark.parametrize("sort_mode", ["presort", "full", "bands", "onesweep"])
@pytest.mark.parametrize("name", CASES)
def test_binning(name, sort_mode):
    sc, cam, cfg, _, g = _run(name, sort_mode)
    tx, ty = oracle.tiles(cam, ocfg_of(cfg))
    check_binning(g, (tx, ty))
    log(f"[P2] {name} {sort_mode}: I={g['I']} bit-exact")


@pytest.mark.parametrize("name", CASES)
def test_forward(name):
    sc, cam, cfg, _, g = _run(name)
    emax, nguard, _ = check_forward(g, cam, cfg)
    log(f"[P3] {name}: max-abs {emax:.2e}, guard pixels {nguard}")


@pytest.mark.parametrize("name", CASES)
def test_backward(name):
    sc, cam, cfg, dimg, g = _run(name)
    oc = ocfg_of(cfg)
    r9 = rec9(g["splat"])
    ref_f = oracle.render_fwd(r9, g["vals"], g["ranges"], cam.width, cam.height, oc)
    g9 = oracle.render_bwd(r9, g["vals"], g["ranges"], cam.width, cam.height, oc,
                           dimg.astype(np.float64))
    tx, _ = oracle.tiles(cam, oc)
    excl = guard_records(ref_f, g["ncontrib"][0], g["ranges"], g["vals"], cfg.tile, tx)
    mask = np.ones(sc.n, bool)
    mask[excl] = False
    w2 = rel_check(g["grad2d"], g9, "grad2d", mask)
    # projection backward from the GPU's 2D gradients
    ref_p = oracle.project_bwd(sc, cam32(cam), oc, g["grad2d"].astype(np.float64))
    worst = {}
    for k in ("means", "scales", "quats", "opacities", "sh"):
        gk, rk = g["grads"][k], ref_p[k]
        gk = gk.reshape(-1, sc.n).T if gk.ndim > 1 else gk
        rk = rk.reshape(-1, sc.n).T if rk.ndim > 1 else rk
        worst[k] = rel_check(gk, rk, k, mask & (g["tc"] > 0))
    log(f"[P4] {name}: grad2d {w2:.2e} x bound, params {worst}, excluded {excl.size}")
