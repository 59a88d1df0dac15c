"""The counting forward (tile_work given) against the oracle: per tile, the
entries its pixels evaluate until they stop and the entries they blend
(the work of Algorithm 1 with the blending of the Background section) equal
the sums of the oracle's per-pixel counts on the GPU's records and lists,
bit-exactly on every tile without a guard pixel; its image, T_final and
n_contrib equal the timed launch's exactly. 3DGS at 8x8, 16x16 (two launch
shapes) and 32x32 tiles on ragged images, 3DGUT and LinPrim."""
import numpy as np
import pytest
import torch

import oracle
from gpu_util import cam32, log, ocfg_of, rec9
from paper_2606_11529_amd import renderer as R
from synth import camera_look_at, scene_clusters

pytestmark = pytest.mark.gpu

CASES = {
    "3dgs_t8": (8, "3dgs", {}),
    "3dgs_t16": (16, "3dgs", {}),
    "3dgs_t16_ppt4_b64_persistent": (16, "3dgs", dict(fwd_ppt=4, lds_batch=64, persistent=True)),
    "3dgs_t32": (32, "3dgs", {}),
    "3dgut_t16": (16, "3dgut", {}),
    "linprim_t16": (16, "linprim", {}),
}


@pytest.mark.parametrize("name", list(CASES))
def test_tile_work_equals_oracle_counts(name):
    tile, method, knobs = CASES[name]
    sc = scene_clusters(6000, seed=8, n_clusters=6, box=1.2, lo=0.005, hi=0.3, sh_degree=1)
    cam = camera_look_at((0.5, -0.2, -3.6), 123, 77)
    cfg = R.Config(tile=tile, sh_degree=1, method=method, **knobs)
    log(f"[work] {name}: n={sc.n} {cam.width}x{cam.height}")
    scene = R.Scene.from_host(sc)
    views = R.Views([scene], [cam], [0], cfg)
    proj = R.xpr_project(views, cfg)
    bins = R.xpr_bin_sort(views, cfg, proj)
    frame = R.xpr_render_fwd(views, cfg, proj, bins)
    tw = torch.full((views.tiles, 2), -1, dtype=torch.int32, device="cuda")
    frame2 = R.xpr_render_fwd(views, cfg, proj, bins, tile_work=tw)
    torch.cuda.synchronize()
    assert torch.equal(frame.image, frame2.image)
    assert torch.equal(frame.T_final, frame2.T_final)
    assert torch.equal(frame.n_contrib, frame2.n_contrib)
    I = bins.count
    vals = bins.vals[:I].cpu().numpy()
    ranges = bins.ranges[:views.tiles].cpu().numpy()
    splat = proj.splat.cpu().numpy()[:views.records]
    oc = ocfg_of(cfg)
    if method == "3dgut":
        ref = oracle.render_fwd_gut(splat[:, :21].astype(np.float64), vals, ranges, cam32(cam), oc)
    elif method == "linprim":
        ref = oracle.render_fwd_lin(splat[:, :17].astype(np.float64), vals, ranges, cam.width,
                                    cam.height, oc)
    else:
        ref = oracle.render_fwd(rec9(splat), vals, ranges, cam.width, cam.height, oc)
    H, W = cam.height, cam.width
    tx, ty = -(-W // tile), -(-H // tile)

    def per_tile(a):
        pad = np.zeros((ty * tile, tx * tile), np.int64)
        pad[:H, :W] = a
        return pad.reshape(ty, tile, tx, tile).sum(axis=(1, 3)).ravel()

    got = tw.cpu().numpy().astype(np.int64)
    g_tiles = per_tile(ref["guard"].astype(np.int64)) > 0
    ok = ~g_tiles
    assert np.array_equal(got[ok, 0], per_tile(ref["neval"])[ok]), "evaluated entries differ"
    assert np.array_equal(got[ok, 1], per_tile(ref["nblend"])[ok]), "blended entries differ"
    assert np.all(got >= 0)
    log(f"[work] {name}: {int(ok.sum())} tiles exact ({int(g_tiles.sum())} with guard pixels), "
        f"evaluated {got[:, 0].sum()}, blended {got[:, 1].sum()}, pairs {I}")
