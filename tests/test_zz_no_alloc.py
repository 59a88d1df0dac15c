"""xpr_render_bwd_noalloc (the backward with the library's static device
scratch, for callers that cannot allocate) against xpr_render_bwd (the
existing entry point, 2D gradients in a caller-owned buffer) through the
C-ABI: two calls in a row, the second with a smaller batch, each equal to
the existing entry point's parameter gradients within the gradient
tolerance (float atomics vary the last bits); with accumulate the result
adds to what the buffers held. Nothing is allocated on the device by the
call itself. For 3DGS, and for 3DGUT and LinPrim (64 bytes of scratch per
record)."""
import numpy as np
import pytest
import torch

from gpu_util import log, rel_check
from paper_2606_11529_amd import renderer as R
from synth import camera_look_at, scene_clusters

pytestmark = pytest.mark.gpu


def _forward(n, W, H, seed, method):
    sc = scene_clusters(n, seed=seed, n_clusters=8, box=1.3, lo=0.005, hi=0.25, sh_degree=3)
    cam = camera_look_at((0.4, -0.3, -3.8), W, H)
    cfg = R.Config(sh_degree=3, method=method)
    scene = R.Scene.from_host(sc)
    views = R.Views([scene], [cam], [0], cfg)
    proj = R.xpr_project(views, cfg)
    bins = R.xpr_bin_sort(views, cfg, proj)
    frame = R.xpr_render_fwd(views, cfg, proj, bins)
    g = torch.Generator(device="cuda")
    g.manual_seed(seed)
    dimg = torch.randn(3 * W * H, generator=g, device="cuda") / (3 * W * H)
    return scene, views, cfg, proj, bins, frame, dimg


def _compare(got, ref, n, tag):
    worst = {}
    for k in ("means", "scales", "quats", "opacities", "sh"):
        gk = got[k].cpu().numpy().astype(np.float64)
        rk = ref[k].cpu().numpy().astype(np.float64)
        gk = gk.reshape(-1, n).T if gk.ndim > 1 else gk
        rk = rk.reshape(-1, n).T if rk.ndim > 1 else rk
        worst[k] = rel_check(gk, rk, f"{tag} {k}")
    return worst


@pytest.mark.parametrize("method", ["3dgs", "3dgut", "linprim"])
def test_noalloc_equals_existing_entry_point_on_two_calls(method):
    for call, (n, W, H, seed) in enumerate([(40_000, 320, 240, 1), (9_000, 150, 97, 2)]):
        scene, views, cfg, proj, bins, frame, dimg = _forward(n, W, H, seed, method)
        ref = R.xpr_render_bwd(views, cfg, proj, bins, frame, dimg)[0][0]
        got = scene.zeros_like_grads()
        for t in got.values():
            t.fill_(7.0)   # overwritten (accumulate = 0)
        torch.cuda.synchronize()
        before = torch.cuda.memory_allocated()
        R.xpr_render_bwd_noalloc(views, cfg, proj, bins, frame, dimg, [got])
        torch.cuda.synchronize()
        assert torch.cuda.memory_allocated() == before
        worst = _compare(got, ref, n, f"call {call}")
        log(f"[noalloc] {method} call {call}: n={n} {W}x{H}, I={bins.count}, worst {worst}")
    # accumulate: adds the gradient to the buffers' contents
    acc = {k: v.clone() for k, v in got.items()}
    R.xpr_render_bwd_noalloc(views, cfg, proj, bins, frame, dimg, [acc], accumulate=True)
    torch.cuda.synchronize()
    _compare({k: acc[k] - got[k] for k in acc}, ref, n, "accumulate")
