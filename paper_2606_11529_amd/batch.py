"""Batched rendering of many views in one launch per stage, with optional
HIP-graph capture of the whole training step.

All views of a batch (uneven resolutions, one or several scenes) share one
projection launch, one binning (a single key space over all views' tiles),
one compositing launch over all tiles (longest lists first, optionally a
persistent grid) and one backward; the projection backward sums the
gradients of every view of a scene inside its kernel. Buffers are sized once
from a profiling pass (the paper's hyperparameter selection also profiles
the views it will render to fix its static sizes), so the step reads nothing
back and can be captured as a graph; after a replay ``overflowed()`` tells
whether the pair count outgrew the capacity (then ``resize`` and capture
again).
"""
from __future__ import annotations

import dataclasses
from typing import List, Optional, Sequence

import torch

from . import renderer as R


class BatchRenderer:
    def __init__(self, scenes: Sequence[R.Scene], cams: Sequence, view_scene: Sequence[int],
                 cfg: R.Config, targets: Optional[Sequence[torch.Tensor]] = None,
                 cap_margin: float = 1.15):
        self.scenes = list(scenes)
        self.cams = list(cams)
        self.view_scene = list(view_scene)
        self.cfg = dataclasses.replace(cfg, no_sync=True)
        self.views = R.Views(self.scenes, self.cams, self.view_scene, self.cfg)
        self.dev = self.scenes[0].means.device
        self.ws = R.Workspace()
        self.graph = None
        self.cap_margin = cap_margin
        # profiling pass (host readback allowed here)
        sync_cfg = dataclasses.replace(self.cfg, no_sync=False)
        v0 = R.Views(self.scenes, self.cams, self.view_scene, sync_cfg)
        p0 = R.xpr_project(v0, sync_cfg)
        b0 = R.xpr_bin_sort(v0, sync_cfg, p0, ws=self.ws)
        self.pairs = b0.count
        self._alloc(int(b0.count * cap_margin) + 4096)
        # L1 loss, summed over views of per-view means: dL/dC = sign / (3 H W)
        scale = torch.cat([torch.full((3 * c.width * c.height,), 1.0 / (3 * c.width * c.height),
                                      device=self.dev) for c in self.cams])
        self.scale = scale
        if targets is None:
            self.target = None
        else:
            self.target = torch.cat([t.reshape(-1) for t in targets]).to(self.dev)
        self.diff = torch.empty(3 * self.views.pixels, device=self.dev)
        self.dimage = torch.empty(3 * self.views.pixels, device=self.dev)

    def _alloc(self, capacity: int) -> None:
        v = self.views
        self.capacity = capacity
        self.proj = R.empty_projected(v.records, self.dev)
        self.bins = R.Bins(vals=torch.empty(capacity, dtype=torch.int32, device=self.dev),
                           ranges=torch.empty((max(v.tiles, 1), 2), dtype=torch.int32,
                                              device=self.dev),
                           n_isect=torch.zeros(1, dtype=torch.int64, device=self.dev),
                           capacity=capacity,
                           tile_order=torch.empty(v.tiles + 1, dtype=torch.int32,
                                                  device=self.dev))
        self.frame = R.Frame(torch.empty(3 * v.pixels, device=self.dev),
                             torch.empty(v.pixels, device=self.dev),
                             torch.empty(v.pixels, dtype=torch.int32, device=self.dev))
        self.grad2d = torch.empty((max(v.records, 1), R.grad2d_floats(self.cfg)), device=self.dev)
        self.grads = [s.zeros_like_grads() for s in self.scenes]
        self.graph = None

    def resize(self, capacity: Optional[int] = None) -> None:
        n = int(self.bins.n_isect.item())
        self._alloc(capacity or int(n * self.cap_margin) + 4096)

    # -- one step ------------------------------------------------------------
    def forward(self) -> torch.Tensor:
        R.xpr_project(self.views, self.cfg, out=self.proj)
        R.xpr_bin_sort(self.views, self.cfg, self.proj, capacity=self.capacity, ws=self.ws,
                       out=self.bins, want_order=True)
        R.xpr_render_fwd(self.views, self.cfg, self.proj, self.bins, out=self.frame)
        return self.frame.image

    def backward(self, dimage: torch.Tensor) -> List[dict]:
        R.xpr_render_bwd(self.views, self.cfg, self.proj, self.bins, self.frame, dimage,
                         params=False, grad2d=self.grad2d, ws=self.ws)
        R.xpr_project_bwd(self.views, self.cfg, self.proj, self.grad2d, grads=self.grads)
        return self.grads

    def step(self) -> None:
        """Forward, L1 gradient against the targets (elementwise only: no
        reduction inside the step, so it captures cleanly), backward."""
        self.forward()
        torch.sub(self.frame.image, self.target, out=self.diff)
        torch.sign(self.diff, out=self.dimage)
        self.dimage.mul_(self.scale)
        self.backward(self.dimage)

    def loss(self) -> float:
        return float((self.diff.abs() * self.scale).sum().item())

    # -- graphs --------------------------------------------------------------
    def capture(self) -> None:
        """Capture ``step`` (after one eager warm-up) as a graph."""
        s = torch.cuda.Stream()
        s.wait_stream(torch.cuda.current_stream())
        with torch.cuda.stream(s):
            self.step()
        torch.cuda.current_stream().wait_stream(s)
        torch.cuda.synchronize()
        g = torch.cuda.CUDAGraph()
        with torch.cuda.graph(g):
            self.step()
        self.graph = g

    def run(self) -> None:
        if self.graph is not None:
            self.graph.replay()
        else:
            self.step()

    def overflowed(self) -> bool:
        return int(self.bins.n_isect.item()) > self.capacity

    def image(self, v: int) -> torch.Tensor:
        return self.views.image(self.frame.image, v)


def per_view_step(scene: R.Scene, cam, cfg: R.Config, target: torch.Tensor,
                  ws: Optional[R.Workspace] = None, state: Optional[dict] = None) -> dict:
    """The same step for one view with plain launches (n_views = 1), the
    baseline the batched launch is compared with."""
    state = state if state is not None else {}
    views = state.get("views") or R.Views([scene], [cam], [0], cfg)
    state["views"] = views
    proj = R.xpr_project(views, cfg, out=state.get("proj"))
    bins = R.xpr_bin_sort(views, cfg, proj, ws=ws, out=state.get("bins"))
    frame = R.xpr_render_fwd(views, cfg, proj, bins, out=state.get("frame"))
    dimg = torch.sign(frame.image - target.reshape(-1)) / frame.image.numel()
    if "grad2d" not in state:
        state["grad2d"] = torch.empty((max(scene.n, 1), R.grad2d_floats(cfg)),
                                      device=scene.means.device)
        state["grads"] = [scene.zeros_like_grads()]
    R.xpr_render_bwd(views, cfg, proj, bins, frame, dimg, params=False, grad2d=state["grad2d"],
                     ws=ws)
    R.xpr_project_bwd(views, cfg, proj, state["grad2d"], grads=state["grads"])
    state.update(proj=proj, bins=bins, frame=frame)
    return state
