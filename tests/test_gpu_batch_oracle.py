"""Batched rendering against the FP64 oracle, view by view, at the shape of
the batched workload: two resident scenes, 12 views of uneven size from
256x256 to 1920x1080 (77,782 tiles at 16x16, so global tile ids need 17 bits
and the pair sort runs on 32-bit tile keys), one launch per stage for all
views, run eagerly with index-order grids and as a replayed HIP graph with
persistent grids over the longest-first tile order.

For every view, with the oracle fed that view's slice of the GPU's buffers
(the stage-wise protocol): P1 projection of its records (at the view's
record offset), P2 its span of the global pair list and tile ranges
bit-exact, P3 its image, T_final and n_contrib, P4 its 2D gradients; and the
parameter gradients the batched projection backward sums over the views of
each scene against the sum of the oracle's per-view gradients (Hyperparameter
selection and the shader's trip-count binning are what the batch, its
capacity and its tile order stand in for)."""
import numpy as np
import pytest
import torch

import oracle
from gpu_util import (cam32, check_forward, check_projection, guard_records, log, ocfg_of, rec9,
                      rel_check)
from paper_2606_11529_amd import renderer as R
from paper_2606_11529_amd.batch import BatchRenderer
from synth import random_cameras, scene_clusters

pytestmark = pytest.mark.gpu

SIZES = [(1920, 1080)] * 8 + [(1600, 1064), (1297, 840), (640, 480), (256, 256)]
VIEW_SCENE = [0, 1, 0, 0, 1, 0, 1, 0, 0, 1, 0, 1]

_RUNS = {}


def _run(mode):
    if mode in _RUNS:
        return _RUNS[mode]
    hosts = [scene_clusters(30_000, seed=31), scene_clusters(12_000, seed=32, n_clusters=16)]
    cams = []
    for k, wh in enumerate(SIZES):
        cams += random_cameras(1, 40 + k, wh)
    if mode == "persistent_graph":
        cfg = R.Config(persistent=True, fwd_ppt=1, bwd_lds_batch=64)
    else:
        cfg = R.Config()
    scenes = [R.Scene.from_host(h) for h in hosts]
    g = torch.Generator(device="cuda")
    g.manual_seed(5)
    targets = [torch.rand((3, c.height, c.width), generator=g, device="cuda") for c in cams]
    log(f"[batch-oracle] mode={mode}: {len(cams)} views, scenes {[h.n for h in hosts]}")
    br = BatchRenderer(scenes, cams, VIEW_SCENE, cfg, targets)
    assert br.views.tiles == 77_782 and br.views.tile_bits >= 17
    if mode == "persistent_graph":
        br.capture()
        for rep in range(2):
            junk = torch.randn(1 << 16, device="cuda").sum().item()  # eager work between
            br.run()
            torch.cuda.synchronize()
        log(f"[batch-oracle] 2 graph replays done ({junk:.1f})")
    else:
        br.step()
        torch.cuda.synchronize()
    assert not br.overflowed()
    v = br.views
    n = v.records
    I = int(br.bins.n_isect.item())
    out = dict(
        hosts=hosts, cams=cams, cfg=cfg, views=v, I=I,
        splat=br.proj.splat.cpu().numpy()[:n], depth=br.proj.depth.cpu().numpy()[:n],
        rect=br.proj.rect.cpu().numpy()[:n].astype(np.int32), tc=br.proj.tc.cpu().numpy()[:n],
        vals=br.bins.vals.cpu().numpy()[:I], ranges=br.bins.ranges.cpu().numpy()[:v.tiles],
        image=[v.image(br.frame.image, k).cpu().numpy() for k in range(len(cams))],
        Tfinal=[v.plane(br.frame.T_final, k).cpu().numpy() for k in range(len(cams))],
        ncontrib=[v.plane(br.frame.n_contrib, k).cpu().numpy() for k in range(len(cams))],
        dimage=[v.image(br.dimage, k).cpu().numpy() for k in range(len(cams))],
        grad2d=br.grad2d.cpu().numpy()[:n],
        grads=[{k: t.cpu().numpy() for k, t in gs.items()} for gs in br.grads])
    log(f"[batch-oracle] mode={mode}: I={I} pairs over {v.tiles} tiles")
    _RUNS[mode] = out
    return out


def _view_slice(s, k):
    """View k's records, tiles and pairs: (rec slice, tile slice, the
    view's span of the global pair list)."""
    v = s["views"]
    cam = s["cams"][k]
    nrec = s["hosts"][VIEW_SCENE[k]].n
    r0, t0 = v.rec_off[k], v.tile_off[k]
    tiles = (-(-cam.width // 16)) * (-(-cam.height // 16))
    rg = s["ranges"][t0:t0 + tiles]
    ne = rg[:, 1] > rg[:, 0]
    p0 = int(rg[ne, 0].min()) if ne.any() else 0
    p1 = int(rg[ne, 1].max()) if ne.any() else 0
    return slice(r0, r0 + nrec), slice(t0, t0 + tiles), p0, p1


def _local_gpu(s, k):
    """View k's buffers in the single-view layout the parity helpers take."""
    rs, ts, p0, p1 = _view_slice(s, k)
    rg = s["ranges"][ts].astype(np.int64)
    ne = rg[:, 1] > rg[:, 0]
    loc = np.where(ne[:, None], rg - p0, 0).astype(np.int32)
    return dict(splat=s["splat"][rs], depth=s["depth"][rs], rect=s["rect"][rs], tc=s["tc"][rs],
                I=p1 - p0, vals=(s["vals"][p0:p1] - rs.start).astype(np.int32), ranges=loc,
                keys=None, image=[s["image"][k]], Tfinal=[s["Tfinal"][k]],
                ncontrib=[s["ncontrib"][k]])


MODES = ["plain_eager", "persistent_graph"]


@pytest.mark.parametrize("mode", MODES)
def test_batch_projection_per_view(mode):
    s = _run(mode)
    for k, cam in enumerate(s["cams"]):
        sc = s["hosts"][VIEW_SCENE[k]]
        ng, n = check_projection(sc, cam, s["cfg"], s, rec_off=s["views"].rec_off[k])
        log(f"[P1] view {k} {cam.width}x{cam.height}: {n} records, {ng} guard")


@pytest.mark.parametrize("mode", MODES)
def test_batch_binning_per_view(mode):
    s = _run(mode)
    total = 0
    for k, cam in enumerate(s["cams"]):
        g = _local_gpu(s, k)
        tx, ty = (-(-cam.width // 16)), (-(-cam.height // 16))
        ref = oracle.bin_pairs(g["depth"].astype(np.float64), g["rect"], g["tc"], tx, ty)
        assert ref["I"] == g["I"], (k, ref["I"], g["I"])
        assert np.array_equal(g["vals"], ref["vals"]), f"view {k}: vals differ"
        assert np.array_equal(g["ranges"], ref["ranges"]), f"view {k}: ranges differ"
        total += ref["I"]
    # the views' spans tile the whole list: nothing outside them
    assert total == s["I"]
    log(f"[P2] {mode}: {len(s['cams'])} views, {total} pairs bit-exact")


@pytest.mark.parametrize("mode", MODES)
def test_batch_forward_per_view(mode):
    s = _run(mode)
    for k, cam in enumerate(s["cams"]):
        emax, ng, _ = check_forward(_local_gpu(s, k), cam, s["cfg"])
        log(f"[P3] {mode} view {k} {cam.width}x{cam.height}: max-abs {emax:.2e}, guard {ng}")


@pytest.mark.parametrize("mode", MODES)
def test_batch_gradients_summed_over_views(mode):
    s = _run(mode)
    cfg = s["cfg"]
    oc = ocfg_of(cfg)
    hosts = s["hosts"]
    ref_sum = [None, None]
    keep = [np.ones(h.n, bool) for h in hosts]
    for k, cam in enumerate(s["cams"]):
        sid = VIEW_SCENE[k]
        g = _local_gpu(s, k)
        r9 = rec9(g["splat"])
        dimg = s["dimage"][k].astype(np.float64)
        ref_f = oracle.render_fwd(r9, g["vals"], g["ranges"], cam.width, cam.height, oc)
        g9 = oracle.render_bwd(r9, g["vals"], g["ranges"], cam.width, cam.height, oc, dimg)
        tx = -(-cam.width // 16)
        excl = guard_records(ref_f, g["ncontrib"][0], g["ranges"], g["vals"], cfg.tile, tx)
        mask = np.ones(hosts[sid].n, bool)
        mask[excl] = False
        keep[sid][excl] = False
        rs = _view_slice(s, k)[0]
        w2 = rel_check(s["grad2d"][rs], g9, f"grad2d view {k}", mask)
        # parameter gradients of this view from the GPU's 2D gradients,
        # summed per scene like the batched projection backward
        ref_p = oracle.project_bwd(hosts[sid], cam32(cam), oc, s["grad2d"][rs].astype(np.float64))
        ref_sum[sid] = ref_p if ref_sum[sid] is None else \
            {kk: ref_sum[sid][kk] + ref_p[kk] for kk in ref_p}
        log(f"[P4] {mode} view {k}: grad2d {w2:.2e} x bound, {excl.size} excluded, |dimg| "
            f"{np.abs(dimg).max():.1e}")
    for sid, h in enumerate(hosts):
        worst = {}
        for name in ("means", "scales", "quats", "opacities", "sh"):
            gk, rk = s["grads"][sid][name], ref_sum[sid][name]
            gk = gk.reshape(-1, h.n).T if gk.ndim > 1 else gk
            rk = rk.reshape(-1, h.n).T if rk.ndim > 1 else rk
            worst[name] = rel_check(gk, rk, f"scene {sid} {name}", keep[sid])
        log(f"[P4] {mode} scene {sid}: summed over views {worst}")
