"""Serving loop: continuous batching of view requests over resident scenes.

Scenes stay resident in HBM. Requests (scene, camera) queue in arrival
order. Device memory for batches comes from one pool of ``budget_bytes``
allocated when the server starts: a batch is admitted only when every
buffer it will use (projected records, pair list, tile ranges, sort
workspace, image planes) has been placed in the pool, so the serving loop's
device memory never exceeds the resident scenes plus the budget. Whenever a
stream slot is free the scheduler forms one batch of up to ``max_views``
views of any scenes and sizes: the queue's prefix (policy ``fifo``, the
default), or the oldest queued request and the next queued requests of its
resolution (policy ``size_class``), as long as the batch still fits the
pool. On the four-scene workload the prefix sustains more frames per
second, so it is the default. A batch runs the
four stages as one batched launch each on its own stream, so batches overlap
on the device; requests arriving meanwhile are admitted as soon as a slot
and memory free up. Each request's image does not depend on what it was
batched with (every view is rendered independently inside the batched
launch).

The pair list is sized from a learned pairs-per-pixel rate per scene, fed
back from the exact pair count of every finished view (its span of the tile
ranges). A batch whose pairs outgrow that capacity is run again with the
exact count, placed in the pool before any new batch; a batch that could
never fit the pool is rejected.

The scheduling policy (pool, admission, batching, accounting) is host logic
in ``Pool`` and ``Scheduler`` and runs against an executor interface:
``GpuExecutor`` drives the HIP path; tests can drive the scheduler with a
host-side executor.
"""
from __future__ import annotations

import collections
import dataclasses
import time
from typing import Callable, Dict, List, Optional, Sequence

# Bytes per unit of the per-batch device buffers, for the scheduler's own
# estimate when no executor-specific sizer is given: record 48 B splat + 4
# depth + 8 rect + 4 count; pair 4 B value plus about 14 B of sort workspace;
# pixel 3x4 B image + 4 B T_final + 4 B n_contrib.
BYTES_PER_RECORD = 64 + 20
BYTES_PER_PAIR = 18
BYTES_PER_PIXEL = 20
ALIGN = 256


def align(n: int) -> int:
    return (int(n) + ALIGN - 1) // ALIGN * ALIGN


class Pool:
    """First-fit allocator over the byte range [0, size) of one device
    buffer; blocks are ALIGN-aligned, freed blocks coalesce with their
    neighbours."""

    def __init__(self, size: int):
        self.size = int(size) // ALIGN * ALIGN
        self.free: List[List[int]] = [[0, self.size]] if self.size > 0 else []
        self.live: Dict[int, int] = {}

    @property
    def used(self) -> int:
        return sum(self.live.values())

    def largest_free(self) -> int:
        return max((n for _, n in self.free), default=0)

    def alloc(self, nbytes: int) -> Optional[int]:
        n = align(max(nbytes, 1))
        for blk in self.free:
            if blk[1] >= n:
                off = blk[0]
                blk[0] += n
                blk[1] -= n
                if blk[1] == 0:
                    self.free.remove(blk)
                self.live[off] = n
                return off
        return None

    def release(self, off: int) -> None:
        n = self.live.pop(off)
        self.free.append([off, n])
        self.free.sort()
        merged: List[List[int]] = []
        for b in self.free:
            if merged and merged[-1][0] + merged[-1][1] == b[0]:
                merged[-1][1] += b[1]
            else:
                merged.append(b)
        self.free = merged


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
    failed: bool = False
    state: object = None

    @property
    def latency(self) -> float:
        return self.t_done - self.t_arrival

    @property
    def pixels(self) -> int:
        return self.cam.width * self.cam.height

    @property
    def size_class(self) -> tuple:
        return (self.cam.width, self.cam.height)


class PairEstimator:
    """Tile-Gaussian pairs per pixel, per scene, learned from finished
    views (starts from a conservative prior)."""

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
    offset: int = -1      # the job's block in the pool


class Scheduler:
    """Admission into batches from a memory pool and a slot count.

    ``sizer(requests, capacity)`` returns the device bytes one batch of
    these requests with a pair list of ``capacity`` entries uses (the
    executor's exact layout); the default is an additive per-request
    estimate."""

    def __init__(self, scene_sizes: Dict[int, int], budget_bytes: int, max_views: int = 8,
                 slots: int = 2, estimator: Optional[PairEstimator] = None,
                 policy: str = "fifo",
                 sizer: Optional[Callable[[List[Request], int], int]] = None):
        if policy not in ("fifo", "size_class"):
            raise ValueError(f"unknown policy {policy!r}")
        self.scene_sizes = dict(scene_sizes)
        self.budget = int(budget_bytes)
        self.pool = Pool(self.budget)
        self.max_views = int(max_views)
        self.slots = int(slots)
        self.policy = policy
        self.est = estimator or PairEstimator()
        self.sizer = sizer or self._additive_bytes
        self.queue: collections.deque = collections.deque()
        self.in_flight: List[Job] = []
        self.reruns: collections.deque = collections.deque()
        self.rejected: List[Request] = []
        self.n_reruns = 0

    @property
    def used(self) -> int:
        return self.pool.used

    def _additive_bytes(self, reqs: List[Request], capacity: int) -> int:
        per = [align(self.scene_sizes[r.scene_id] * BYTES_PER_RECORD + r.pixels * BYTES_PER_PIXEL)
               for r in reqs]
        return sum(per) + align(capacity * BYTES_PER_PAIR)

    def capacity_of(self, reqs: List[Request]) -> int:
        return sum(self.est.estimate(r.scene_id, r.pixels) for r in reqs)

    def job_bytes(self, reqs: List[Request], capacity: int) -> int:
        return align(self.sizer(reqs, capacity))

    def request_bytes(self, req: Request) -> int:
        return self.job_bytes([req], self.capacity_of([req]))

    def submit(self, req: Request) -> None:
        if self.request_bytes(req) > self.pool.size:
            req.failed = True
            self.rejected.append(req)  # can never fit, even alone
            return
        self.queue.append(req)

    def free_slots(self) -> List[int]:
        busy = {j.slot for j in self.in_flight}
        return [s for s in range(self.slots) if s not in busy]

    def _place(self, job: Job, slot: int) -> bool:
        off = self.pool.alloc(job.bytes)
        if off is None:
            return False
        job.offset, job.slot = off, slot
        self.in_flight.append(job)
        return True

    def next_job(self) -> Optional[Job]:
        """A job for the lowest free slot: first a job to run again with a
        larger pair list, else a new batch (see the module notes). None if
        nothing fits now."""
        free = self.free_slots()
        if not free:
            return None
        if self.reruns:
            job = self.reruns[0]
            job.bytes = self.job_bytes(job.requests, job.capacity)
            if job.bytes > self.pool.size:
                self.reruns.popleft()
                for r in job.requests:
                    r.failed = True
                    self.rejected.append(r)
                return self.next_job()
            if not self._place(job, free[0]):
                return None
            self.reruns.popleft()
            return job
        if not self.queue:
            return None
        room = self.pool.largest_free()
        head = self.queue[0]
        reqs: List[Request] = []
        for req in self.queue:
            if len(reqs) == self.max_views:
                break
            if self.policy == "size_class" and req.size_class != head.size_class:
                continue
            trial = reqs + [req]
            if self.job_bytes(trial, self.capacity_of(trial)) > room:
                break
            reqs.append(req)
        if not reqs:
            return None
        job = Job(requests=reqs, bytes=self.job_bytes(reqs, self.capacity_of(reqs)),
                  capacity=self.capacity_of(reqs))
        if not self._place(job, free[0]):
            return None
        taken = {id(r) for r in reqs}
        self.queue = collections.deque(r for r in self.queue if id(r) not in taken)
        return job

    def rerun(self, job: Job) -> None:
        """The job's pairs outgrew its list: release its block and queue it
        to run again (job.capacity has been raised by the executor)."""
        self.in_flight.remove(job)
        self.pool.release(job.offset)
        job.offset = -1
        job.handle = None
        self.n_reruns += 1
        self.reruns.append(job)

    def finish(self, job: Job) -> None:
        self.in_flight.remove(job)
        self.pool.release(job.offset)
        for r in job.requests:
            if r.pairs >= 0:
                self.est.update(r.scene_id, r.pixels, r.pairs)


class _PoolSlice:
    """The sort workspace of one job: a fixed slice of the pool (the
    renderer asks it for a buffer of at least the bytes it needs)."""

    def __init__(self, t):
        self.t = t

    def get(self, name, nbytes, device):
        if self.t.numel() < nbytes:
            raise RuntimeError(f"workspace slice of {self.t.numel()} B < {nbytes} B")
        return self.t


class GpuExecutor:
    """Runs a batch through the C-ABI on the stream of its slot, with every
    buffer of the batch carved out of one device pool of the budget's size
    (allocated once, here)."""

    def __init__(self, scenes: Dict[int, "object"], cfg, n_slots: int, budget_bytes: int,
                 keep_images: bool = True, keep_state: bool = False):
        import torch

        from . import renderer as R
        self.R = R
        self.torch = torch
        self.scenes = scenes
        self.cfg = dataclasses.replace(cfg, no_sync=True)
        dev = next(iter(scenes.values())).means.device
        self.pool = torch.empty(max(int(budget_bytes) // ALIGN * ALIGN, ALIGN), dtype=torch.uint8,
                                device=dev)
        # default-priority streams, one per slot
        self.streams = [torch.cuda.Stream() for _ in range(n_slots)]
        self.keep_images = keep_images
        # keep_state: each request also gets host copies of the records and
        # pair lists its view was rendered from (for checking a served image
        # against a reference renderer on exactly its inputs)
        self.keep_state = keep_state

    def _views(self, reqs: Sequence[Request]):
        ids = sorted({r.scene_id for r in reqs})
        local = {sid: k for k, sid in enumerate(ids)}
        return self.R.Views([self.scenes[s] for s in ids], [r.cam for r in reqs],
                            [local[r.scene_id] for r in reqs], self.cfg)

    def layout(self, views, capacity: int):
        """(name, dtype, shape) of every buffer of a batch, and the bytes
        they take at ALIGN-aligned offsets."""
        R, torch = self.R, self.torch
        L = R.L
        nrec, nt, npx = max(views.records, 1), max(views.tiles, 1), max(views.pixels, 1)
        order = self.cfg.persistent or self.cfg.tile_order
        bufs = [("splat", torch.float32, (nrec, R.splat_floats(self.cfg))),
                ("depth", torch.float32, (nrec,)), ("rect", torch.int16, (nrec, 4)),
                ("tc", torch.int32, (nrec,)), ("vals", torch.int32, (max(capacity, 1),)),
                ("ranges", torch.int32, (nt, 2)), ("n_isect", torch.int64, (1,)),
                ("image", torch.float32, (3 * npx,)), ("T_final", torch.float32, (npx,)),
                ("n_contrib", torch.int32, (npx,)),
                ("ws", torch.uint8, (max(L.xpr_bin_sort_workspace(views.c, views.cfg_c,
                                                                   capacity), 1),))]
        if order:
            bufs.append(("tile_order", torch.int32, (nt + 1,)))
        total = 0
        for _, dt, shape in bufs:
            n = 1
            for d in shape:
                n *= d
            total += align(n * torch.tensor([], dtype=dt).element_size())
        return bufs, total

    def job_bytes(self, reqs: List[Request], capacity: int) -> int:
        return self.layout(self._views(reqs), capacity)[1]

    def launch(self, job: Job):
        R, torch = self.R, self.torch
        views = self._views(job.requests)
        bufs, total = self.layout(views, job.capacity)
        if job.offset < 0 or total > job.bytes:
            raise RuntimeError(f"job needs {total} B, its pool block holds {job.bytes} B")
        t = {}
        off = job.offset
        for name, dt, shape in bufs:
            es = torch.tensor([], dtype=dt).element_size()
            n = 1
            for d in shape:
                n *= d
            t[name] = self.pool[off:off + n * es].view(dt).view(shape)
            off += align(n * es)
        proj = R.Projected(t["splat"], t["depth"], t["rect"], t["tc"])
        bins = R.Bins(vals=t["vals"], ranges=t["ranges"], n_isect=t["n_isect"],
                      capacity=job.capacity, tile_order=t.get("tile_order"))
        frame = R.Frame(t["image"], t["T_final"], t["n_contrib"])
        st = self.streams[job.slot]
        st.wait_stream(torch.cuda.current_stream())
        with torch.cuda.stream(st):
            R.xpr_project(views, self.cfg, out=proj)
            R.xpr_bin_sort(views, self.cfg, proj, capacity=job.capacity, ws=_PoolSlice(t["ws"]),
                           out=bins)
            R.xpr_render_fwd(views, self.cfg, proj, bins, out=frame)
            ev = torch.cuda.Event()
            ev.record(st)
        return dict(views=views, proj=proj, bins=bins, frame=frame, event=ev, stream=st)

    def done(self, handle) -> bool:
        return handle["event"].query()

    def collect(self, job: Job, handle) -> bool:
        """Fill the requests' results (images copied to host memory, so
        nothing of a finished batch stays on the device) and their exact
        pair counts; False if the pair list was too small (the job must run
        again with the exact capacity now in job.capacity)."""
        views, bins, frame = handle["views"], handle["bins"], handle["frame"]
        n = int(bins.n_isect.item())
        if n > bins.capacity:
            job.capacity = n
            return False
        # pairs of view v: the sum of its tiles' range lengths (copied to
        # host memory first: nothing is allocated on the device here)
        rg = bins.ranges[:views.tiles].to("cpu")
        lens = (rg[:, 1] - rg[:, 0]).to(self.torch.int64)
        for v, r in enumerate(job.requests):
            t0 = views.tile_off[v]
            t1 = views.tile_off[v + 1] if v + 1 < views.n_views else views.tiles
            r.pairs = int(lens[t0:t1].sum())
            if self.keep_images:
                r.image = views.image(frame.image, v).to("cpu")
            if self.keep_state:
                r0 = views.rec_off[v]
                r1 = r0 + views.scenes[views.view_scene[v]].n
                seg = rg[t0:t1].numpy()
                ne = seg[:, 1] > seg[:, 0]
                p0 = int(seg[ne, 0].min()) if ne.any() else 0
                p1 = int(seg[ne, 1].max()) if ne.any() else 0
                proj = handle["proj"]
                r.state = dict(
                    splat=proj.splat[r0:r1].to("cpu").numpy(),
                    depth=proj.depth[r0:r1].to("cpu").numpy(),
                    rect=proj.rect[r0:r1].to("cpu").numpy(), tc=proj.tc[r0:r1].to("cpu").numpy(),
                    vals=(bins.vals[p0:p1].to("cpu").numpy() - r0),
                    ranges=(seg - p0) * ne[:, None],
                    T_final=views.plane(frame.T_final, v).to("cpu").numpy(),
                    n_contrib=views.plane(frame.n_contrib, v).to("cpu").numpy())
        return True


class Server:
    """Continuous-batching server over resident scenes."""

    def __init__(self, scenes: Dict[int, "object"], cfg, budget_bytes: int, max_views: int = 8,
                 slots: int = 2, executor=None, clock: Callable[[], float] = time.perf_counter,
                 keep_images: bool = True, policy: str = "fifo",
                 estimator: Optional[PairEstimator] = None, keep_state: bool = False):
        self.exec = executor or GpuExecutor(scenes, cfg, slots, budget_bytes,
                                            keep_images=keep_images, keep_state=keep_state)
        self.sched = Scheduler({k: s.n for k, s in scenes.items()}, budget_bytes, max_views,
                               slots, estimator=estimator, policy=policy,
                               sizer=getattr(self.exec, "job_bytes", None))
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
                    self.sched.rerun(job)
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
        return not self.sched.queue and not self.sched.in_flight and not self.sched.reruns

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
