"""The backward with heavy tiles split into four 16x4 bands (bwd_split_walk)
against the oracle's analytic backward (P4, 1e-3 relative per tensor) and
against the unsplit launch, with every tile split (threshold 1), a mixed
threshold, and tile order; images are not touched by the backward."""
import numpy as np
import pytest

import oracle
from gpu_util import cam32, guard_records, log, ocfg_of, rec9, rel_check, run_gpu
from paper_2606_11529_amd import renderer as R
from synth import camera_look_at, scene_clusters

pytestmark = pytest.mark.gpu

_CASE = {}


def _case():
    if not _CASE:
        sc = scene_clusters(60_000, seed=13, n_clusters=6, box=1.0, lo=0.004, hi=0.12)
        cam = camera_look_at((0.3, -0.2, -3.2), 211, 147)
        rng = np.random.default_rng(4)
        dimg = (rng.normal(size=(3, cam.height, cam.width)) /
                (3 * cam.width * cam.height)).astype(np.float32)
        _CASE.update(sc=sc, cam=cam, dimg=dimg,
                     ref=run_gpu(sc, cam, R.Config(bwd_ppt=4), dimgs=[dimg]))
    return _CASE


@pytest.mark.parametrize("split,order", [(1, False), (1, True), (200, False), (200, True)])
def test_split_backward_matches_unsplit_and_oracle(split, order):
    c = _case()
    sc, cam, dimg, ref = c["sc"], c["cam"], c["dimg"], c["ref"]
    cfg = R.Config(bwd_ppt=4, bwd_split_walk=split, tile_order=order)
    g = run_gpu(sc, cam, cfg, dimgs=[dimg])
    assert np.array_equal(g["vals"], ref["vals"])
    nc = g["ncontrib"][0]
    H, W = nc.shape
    tx, ty = -(-W // 16), -(-H // 16)
    pad = np.zeros((ty * 16, tx * 16), np.int64)
    pad[:H, :W] = nc
    walks = pad.reshape(ty, 16, tx, 16).max(axis=(1, 3))
    nsplit = int((walks >= split).sum())
    assert nsplit > 0 and (split == 1 or nsplit < walks.size)
    # the unsplit launch: the same sums in another order
    rel_check(g["grad2d"], ref["grad2d"], "grad2d vs unsplit", tol=1e-4)
    for k in g["grads"]:
        a, b = g["grads"][k], ref["grads"][k]
        assert np.abs(a - b).max() <= 1e-4 * np.abs(b).max() + 1e-30, k
    # the oracle
    oc = ocfg_of(cfg)
    r9 = rec9(g["splat"])
    ref_f = oracle.render_fwd(r9, g["vals"], g["ranges"], W, H, oc)
    g9 = oracle.render_bwd(r9, g["vals"], g["ranges"], W, H, oc, dimg.astype(np.float64))
    excl = guard_records(ref_f, nc, g["ranges"], g["vals"], 16, tx)
    mask = np.ones(sc.n, bool)
    mask[excl] = False
    w = rel_check(g["grad2d"], g9, "grad2d", mask)
    ref_p = oracle.project_bwd(sc, cam32(cam), oc, g["grad2d"].astype(np.float64))
    worst = {}
    for k in ("means", "scales", "quats", "opacities", "sh"):
        gk, rk = g["grads"][k], ref_p[k]
        gk = gk.reshape(-1, sc.n).T if gk.ndim > 1 else gk
        rk = rk.reshape(-1, sc.n).T if rk.ndim > 1 else rk
        worst[k] = rel_check(gk, rk, k, mask & (g["tc"] > 0))
    log(f"[split] walk >= {split} order={order}: {nsplit} of {walks.size} tiles split "
        f"(longest walk {walks.max()}), grad2d {w:.2e} x bound, params {worst}")
