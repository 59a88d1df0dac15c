"""Whole-frame parity of the 3DGUT and LinPrim paths (LinPrim also with its
tile cull) at the full benchmark size (3M primitives, SH degree 3,
1600x1064, 16x16 tiles), on the camera of the eight whose densest tile
walks furthest, against the FP64 oracle, each stage fed the GPU's previous
stage: every primitive's projection (P1), the whole pair list and every
tile range bit-exact (P2; with the cull, the oracle's cull of every pair on
the GPU's float32 records), every pixel's colour, T_final and n_contrib
(P3), and every record's 16 shader-data gradients and every primitive's
parameter gradients (P4). dL/dimage is zero on the guard pixels, so no
decision in the guard band reaches a gradient and P4 covers every record.
The oracle takes about 10 s per frame and method on 16 host cores."""
import functools

import numpy as np
import pytest

import oracle
import test_gpu_gut as GUT
import test_gpu_linprim as LIN
from gpu_util import cam32, check_binning, check_binning_cull, log, ocfg_of, run_gpu
from paper_2606_11529_amd import renderer as R
from synth import random_cameras, scene_clusters

pytestmark = pytest.mark.gpu


@functools.lru_cache(maxsize=1)
def _scene():
    log("[full-m] generating 3M-primitive scene")
    return scene_clusters(3_000_000, seed=0), random_cameras(8, 0, (1600, 1064))[5]


@pytest.mark.parametrize("method,cull", [("3dgut", False), ("linprim", False), ("linprim", True)])
def test_fullsize_method_whole_frame(method, cull):
    sc, cam = _scene()
    cfg = R.Config(sh_degree=3, method=method, tile_cull=cull)
    M = GUT if method == "3dgut" else LIN
    log(f"[full-m] method={method} cull={cull} n={sc.n} {cam.width}x{cam.height}")
    H, W = cam.height, cam.width
    tx, ty = (W + 15) // 16, (H + 15) // 16
    oc = ocfg_of(cfg)
    g0 = run_gpu(sc, cam, cfg)

    # P1: every primitive
    ng = M._check_projection(sc, cam, cfg, g0, np.arange(sc.n))

    # P2: the whole list and every range
    if cull:
        ref_b = check_binning_cull(g0, cam, cfg, (tx, ty))
        assert g0["I"] < int(g0["tc"].astype(np.int64).sum())
    else:
        ref_b = check_binning(g0, (tx, ty))
    log(f"[full-m] {method} cull={cull}: P1 {sc.n} ({ng} guard), P2 I={g0['I']} bit-exact "
        f"(guard pairs {ref_b.get('n_guard', 0)})")

    # P3: every pixel
    emax, ngp = M._check_forward(g0, cam, cfg)

    # P4: dL/dimage zero on the guard pixels, then every record and primitive
    ncol = 21 if method == "3dgut" else 17
    rec = g0["splat"][:, :ncol].astype(np.float64)
    if method == "3dgut":
        ref_f = oracle.render_fwd_gut(rec, g0["vals"], g0["ranges"], cam32(cam), oc)
    else:
        ref_f = oracle.render_fwd_lin(rec, g0["vals"], g0["ranges"], W, H, oc)
    rng = np.random.default_rng(3)
    dimg = rng.normal(size=(3, H, W)).astype(np.float32) / (3 * W * H)
    dimg[:, ref_f["guard"].astype(bool)] = 0.0
    g = run_gpu(sc, cam, cfg, dimgs=[dimg])
    assert np.array_equal(g["vals"], g0["vals"]) and np.array_equal(g["image"][0], g0["image"][0])
    w16, worst, _ = M._backward_check(sc, cam, cfg, g, dimg, exclude_guard=False)
    log(f"[full-m] {method} cull={cull}: P3 {W * H} px max-abs {emax:.2e} ({ngp} guard), "
        f"P4 grad16 {w16:.2e} x bound over all {sc.n} records, params {worst}")
