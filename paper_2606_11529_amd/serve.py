"""Serving loop: continuous batching of view requests over resident scenes.

Scenes stay resident in HBM. Requests (scene, camera) queue in arrival
order; whenever a stream slot is free the scheduler admits queued requests
into one batch while their estimated device memory fits the budget left by
the batches still in flight, up to ``max_views`` views of any resolutions
and scenes. A batch runs the four stages as one batched launch each on its
own stream, so batches overlap on the device; requests arriving meanwhile are
admitted as soon as a slot and memory free up. Each request's image does not
depend on what it was batched with (every view is rendered independently
inside the batched launch).

The scheduling policy (admission, batching, accounting) is host logic in
``Scheduler`` and runs against an executor interface: ``GpuExecutor`` drives
the HIP path; tests can drive the scheduler with a host-side executor.
"""
from __future__ import annotations

import collections
import dataclasses
import time
from typing import Callable, Dict, List, Optional, Sequence

# Bytes per unit of the per-batch device allocations (see GpuExecutor):
# record 48 B splat + 4 depth + 8 rect + 4 count; pair 4 B value plus about
# 14 B of sort workspace (two key buffers, one alternate value buffer and
# histograms); pixel 3x4 B image + 4 B T_final + 4 B n_contrib.
BYTES_PER_RECORD = 64 + 20
BYTES_PER_PAIR = 18
BYTES_PER_PIXEL = 20


@dataclasses.dataclass
class Request:
    rid: int
    scene_id: int
    cam: object
    t_arrival: float
    t_admit: float = -1.0
    t_done: float = -1.0
    image: object = None
    pairs: int = -1

    @property
    def latency(self) -> float:
        return self.t_done - self.t_arrival


class PairEstimator:
    """Tile-Gaussian pairs per pixel, per scene, learned from finished
    batches (starts from a conservative prior)."""

    def __init__(self, prior_per_pixel: float = 40.0, margin: float = 1.3):
        self.rate: Dict[int, float] = {}
        self.prior = prior_per_pixel
        self.margin = margin

    def estimate(self, scene_id: int, pixels: int) -> int:
        r = self.rate.get(scene_id, self.prior)
        return int(r * pixels * self.margin) + 4096

    def update(self, scene_id: int, pixels: int, pairs: int) -> None:
        r = pairs / max(pixels, 1)
        old = self.rate.get(scene_id)
        self.rate[scene_id] = r if old is None else max(r, 0.5 * (old + r))


@dataclasses.dataclass
class Job:
    requests: List[Request]
    bytes: int
    capacity: int
    handle: object = None
    slot: int = -1


class Scheduler:
    """FIFO admission into batches under a memory budget and a slot count."""

    def __init__(self, scene_sizes: Dict[int, int], budget_bytes: int, max_views: int = 8,
                 slots: int = 2, estimator: Optional[PairEstimator] = None):
        self.scene_sizes = dict(scene_sizes)
        self.budget = int(budget_bytes)
        self.max_views = int(max_views)
        self.slots = int(slots)
        self.est = estimator or PairEstimator()
        self.queue: collections.deque = collections.deque()
        self.in_flight: List[Job] = []
        self.used = 0
        self.rejected: List[Request] = []

    def request_bytes(self, req: Request) -> int:
        px = req.cam.width * req.cam.height
        return (self.scene_sizes[req.scene_id] * BYTES_PER_RECORD
                + self.est.estimate(req.scene_id, px) * BYTES_PER_PAIR + px * BYTES_PER_PIXEL)

    def submit(self, req: Request) -> None:
        if self.request_bytes(req) > self.budget:
            self.rejected.append(req)  # can never fit, even alone
            return
        self.queue.append(req)

    def free_slots(self) -> List[int]:
        busy = {j.slot for j in self.in_flight}
        return [s for s in range(self.slots) if s not in busy]

    def next_job(self) -> Optional[Job]:
        """Admit the longest FIFO prefix that fits the free memory and the
        view limit, into the lowest free slot. None if nothing fits now."""
        free = self.free_slots()
        if not self.queue or not free:
            return None
        reqs, total, cap = [], 0, 0
        for req in self.queue:
            if len(reqs) == self.max_views:
                break
            b = self.request_bytes(req)
            if self.used + total + b > self.budget:
                break
            reqs.append(req)
            total += b
            cap += self.est.estimate(req.scene_id, req.cam.width * req.cam.height)
        if not reqs:
            return None
        for _ in reqs:
            self.queue.popleft()
        job = Job(requests=reqs, bytes=total, capacity=cap, slot=free[0])
        self.used += total
        self.in_flight.append(job)
        return job

    def finish(self, job: Job) -> None:
        self.in_flight.remove(job)
        self.used -= job.bytes
        for r in job.requests:
            if r.pairs >= 0:
                self.est.update(r.scene_id, r.cam.width * r.cam.height, r.pairs)


class GpuExecutor:
    """Runs a batch through the C-ABI on the stream of its slot."""

    def __init__(self, scenes: Dict[int, "object"], cfg, n_slots: int, keep_images: bool = True):
        import torch

        from . import renderer as R
        self.R = R
        self.torch = torch
        self.scenes = scenes
        self.cfg = dataclasses.replace(cfg, no_sync=True)
        # default-priority streams, one per slot
        self.streams = [torch.cuda.Stream() for _ in range(n_slots)]
        self.ws = [R.Workspace() for _ in range(n_slots)]
        self.keep_images = keep_images

    def launch(self, job: Job):
        R, torch = self.R, self.torch
        ids = sorted({r.scene_id for r in job.requests})
        local = {sid: k for k, sid in enumerate(ids)}
        st = self.streams[job.slot]
        st.wait_stream(torch.cuda.current_stream())
        with torch.cuda.stream(st):
            views = R.Views([self.scenes[s] for s in ids], [r.cam for r in job.requests],
                            [local[r.scene_id] for r in job.requests], self.cfg)
            proj = R.xpr_project(views, self.cfg)
            bins = R.xpr_bin_sort(views, self.cfg, proj, capacity=job.capacity, ws=self.ws[job.slot])
            frame = R.xpr_render_fwd(views, self.cfg, proj, bins)
            ev = torch.cuda.Event()
            ev.record(st)
        return dict(views=views, proj=proj, bins=bins, frame=frame, event=ev, stream=st)

    def done(self, handle) -> bool:
        return handle["event"].query()

    def collect(self, job: Job, handle) -> bool:
        """Fill the requests' results; False if the pair capacity was too
        small (the job must be run again with a larger capacity)."""
        views, bins, frame = handle["views"], handle["bins"], handle["frame"]
        n = int(bins.n_isect.item())
        if n > bins.capacity:
            job.capacity = int(n * 1.1) + 4096
            return False
        total_px = sum(r.cam.width * r.cam.height for r in job.requests)
        for v, r in enumerate(job.requests):
            px = r.cam.width * r.cam.height
            r.pairs = int(n * px / total_px)
            if self.keep_images:
                r.image = views.image(frame.image, v).clone()
        return True


class Server:
    """Continuous-batching server over resident scenes."""

    def __init__(self, scenes: Dict[int, "object"], cfg, budget_bytes: int, max_views: int = 8,
                 slots: int = 2, executor=None, clock: Callable[[], float] = time.perf_counter,
                 keep_images: bool = True):
        self.sched = Scheduler({k: s.n for k, s in scenes.items()}, budget_bytes, max_views,
                               slots)
        self.exec = executor or GpuExecutor(scenes, cfg, slots, keep_images=keep_images)
        self.clock = clock
        self.done: List[Request] = []
        self._rid = 0

    def submit(self, scene_id: int, cam, t_arrival: Optional[float] = None) -> Request:
        req = Request(self._rid, scene_id, cam, self.clock() if t_arrival is None else t_arrival)
        self._rid += 1
        self.sched.submit(req)
        return req

    def poll(self) -> int:
        """Retire finished batches, then admit and launch new ones. Returns
        the number of requests completed."""
        n = 0
        for job in list(self.sched.in_flight):
            if job.handle is not None and self.exec.done(job.handle):
                if self.exec.collect(job, job.handle):
                    t = self.clock()
                    for r in job.requests:
                        r.t_done = t
                        self.done.append(r)
                    n += len(job.requests)
                    self.sched.finish(job)
                else:
                    job.handle = self.exec.launch(job)
        while True:
            job = self.sched.next_job()
            if job is None:
                break
            t = self.clock()
            for r in job.requests:
                r.t_admit = t
            job.handle = self.exec.launch(job)
        return n

    def idle(self) -> bool:
        return not self.sched.queue and not self.sched.in_flight

    def drain(self, sleep: float = 0.0) -> None:
        while not self.idle():
            self.poll()
            if sleep:
                time.sleep(sleep)


def replay(server: Server, arrivals: Sequence, scenes_of=None, speed: float = 1.0,
           spin: float = 2e-4) -> float:
    """Feeds (arrival_s, scene_id, camera) requests at their arrival times
    (scaled by ``speed``) and polls the server until all complete. Returns
    the wall time."""
    t0 = server.clock()
    i = 0
    while i < len(arrivals) or not server.idle():
        now = server.clock() - t0
        while i < len(arrivals) and arrivals[i][0] / speed <= now:
            a, sid, cam = arrivals[i]
            server.submit(sid, cam, t_arrival=t0 + a / speed)
            i += 1
        server.poll()
        if spin:
            time.sleep(spin)
    return server.clock() - t0


def latency_stats(reqs: Sequence[Request]) -> dict:
    import numpy as np
    lat = np.array([r.latency for r in reqs]) * 1e3
    return {"n": int(lat.size), "p50_ms": float(np.percentile(lat, 50)),
            "p99_ms": float(np.percentile(lat, 99)), "mean_ms": float(lat.mean()),
            "max_ms": float(lat.max())}
