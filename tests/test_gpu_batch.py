"""Batched multi-view rendering: the graph-captured step replays to the eager
result (several replays with eager work and synchronisation in between), the
batch equals per-view plain launches, render_batch over two scenes equals
render() per view (16 and 32 tiles), and the overflow check works."""
import numpy as np
import pytest
import torch

from gpu_util import log
from paper_2606_11529_amd import renderer as R
from paper_2606_11529_amd.batch import BatchRenderer, per_view_step
from synth import random_cameras, scene_clusters

pytestmark = pytest.mark.gpu


def _setup(n=8000, seed=4, nv=5):
    sc = scene_clusters(n, seed=seed, n_clusters=8, box=1.5)
    cams = random_cameras(nv, seed, [(64, 64), (160, 120), (97, 53), (200, 150)], radius=4.5)
    g = torch.Generator(device="cuda")
    g.manual_seed(1)
    targets = [torch.rand((3, c.height, c.width), generator=g, device="cuda") for c in cams]
    return R.Scene.from_host(sc), cams, targets


@pytest.mark.parametrize("persistent", [False, True])
def test_graph_replays_equal_eager(persistent):
    scene, cams, targets = _setup()
    br = BatchRenderer([scene], cams, [0] * len(cams), R.Config(persistent=persistent), targets)
    br.step()
    torch.cuda.synchronize()
    ref_img = br.frame.image.clone()
    ref_g = {k: v.clone() for k, v in br.grads[0].items()}
    br.capture()
    for rep in range(4):
        junk = torch.randn(4096, device="cuda").sum().item()   # eager work between replays
        br.run()
        torch.cuda.synchronize()
        assert not br.overflowed()
        assert torch.equal(br.frame.image, ref_img), rep
        for k, v in br.grads[0].items():
            scale = ref_g[k].abs().max().item()
            assert (v - ref_g[k]).abs().max().item() <= 1e-4 * scale + 1e-12, (rep, k)
    log(f"[graph] persistent={persistent}: 4 replays equal eager, loss {br.loss():.4f}, {junk:.2f}")


def test_batch_equals_per_view_plain_launches():
    scene, cams, targets = _setup(seed=6)
    br = BatchRenderer([scene], cams, [0] * len(cams), R.Config(), targets)
    br.step()
    torch.cuda.synchronize()
    total = None
    for v, (cam, t) in enumerate(zip(cams, targets)):
        st = per_view_step(scene, cam, R.Config(), t)
        torch.cuda.synchronize()
        assert torch.equal(br.image(v), st["views"].image(st["frame"].image, 0)), v
        g = st["grads"][0]
        total = {k: x.clone() for k, x in g.items()} if total is None else \
            {k: total[k] + g[k] for k in total}
    for k in total:
        scale = total[k].abs().max().item()
        assert (br.grads[0][k] - total[k]).abs().max().item() <= 1e-4 * scale, k


def test_overflow_detected_and_resize():
    scene, cams, targets = _setup(seed=7, nv=3)
    br = BatchRenderer([scene], cams, [0] * len(cams), R.Config(), targets)
    need = br.pairs
    br._alloc(need // 2)
    br.step()
    torch.cuda.synchronize()
    assert br.overflowed()
    br.resize()
    br.step()
    torch.cuda.synchronize()
    assert not br.overflowed() and int(br.bins.n_isect.item()) == need


@pytest.mark.parametrize("tile", [16, 32])
def test_render_batch_equals_single_views(tile):
    # two scenes, views of four sizes; every view equals its own render()
    sa = R.Scene.from_host(scene_clusters(6000, seed=21, n_clusters=6, box=1.4))
    sb = R.Scene.from_host(scene_clusters(3000, seed=22, n_clusters=4, box=1.0, sh_degree=1))
    cams = random_cameras(5, 23, [(64, 64), (160, 120), (97, 53), (200, 150)], radius=4.5)
    vs = [0, 1, 0, 1, 1]
    cfg = R.Config(tile=tile, sh_degree=1)
    images, st = R.render_batch([sa, sb], cams, cfg, view_scene=vs)
    assert len(images) == len(cams)
    for v, cam in enumerate(cams):
        one, _ = R.render([sa, sb][vs[v]], cam, cfg)
        assert images[v].shape == (3, cam.height, cam.width)
        assert torch.equal(images[v], one), v
    log(f"[batch] render_batch tile {tile}: {len(cams)} views, I={st['bins'].count}")
