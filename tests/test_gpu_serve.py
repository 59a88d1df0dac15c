"""Serving on the GPU: requests of several scenes and resolutions batched by
the continuous-batching server (overlapping on two streams, admitted under a
memory budget) return exactly the image each request gets when rendered
alone."""
import numpy as np
import pytest
import torch

from gpu_util import log
from paper_2606_11529_amd import renderer as R
from paper_2606_11529_amd import serve as S
from synth import random_cameras, scene_clusters

pytestmark = pytest.mark.gpu


def test_each_result_same_alone_and_in_the_mix():
    hosts = {0: scene_clusters(20_000, seed=0, n_clusters=8), 1: scene_clusters(60_000, seed=1)}
    scenes = {k: R.Scene.from_host(v) for k, v in hosts.items()}
    cfg = R.Config()
    rng = np.random.default_rng(3)
    res = [(128, 96), (200, 120), (96, 160), (64, 64)]
    cams = random_cameras(24, 11, res)
    sids = rng.integers(0, 2, size=len(cams)).tolist()
    budget = 64 << 20   # forces several batches
    srv = S.Server(scenes, cfg, budget, max_views=6, slots=2)
    reqs = []
    for k, (sid, cam) in enumerate(zip(sids, cams)):
        reqs.append(srv.submit(sid, cam))
        if k % 5 == 4:
            srv.poll()      # later requests arrive while earlier batches run
    srv.drain()
    torch.cuda.synchronize()
    assert len(srv.done) == len(reqs) and not srv.sched.rejected
    for r in reqs:
        img, _ = R.render(scenes[r.scene_id], r.cam, cfg)
        torch.cuda.synchronize()
        assert torch.equal(r.image, img), r.rid
    st = S.latency_stats(srv.done)
    log(f"[serve] {st}")
