"""Host logic of the serving loop (the budget pool, admission by memory,
FIFO and size-class batching, slots, continuous admission, capacity re-run),
driven by a host-side executor with a simulated clock: no GPU involved."""
import dataclasses

import numpy as np
import pytest

from paper_2606_11529_amd import serve as S


@dataclasses.dataclass
class Cam:
    width: int
    height: int


class Clock:
    def __init__(self):
        self.t = 0.0

    def __call__(self):
        return self.t


class FakeExec:
    """Completes a job `latency` seconds after launch; reports `pairs_per_px`
    pairs per pixel (and once, optionally, too many pairs for the capacity)."""

    def __init__(self, clock, latency=0.01, pairs_per_px=10.0, overflow_once=False):
        self.clock, self.latency, self.ppp = clock, latency, pairs_per_px
        self.launched = []
        self.overflow_once = overflow_once

    def launch(self, job):
        self.launched.append([r.rid for r in job.requests])
        return {"ready": self.clock() + self.latency}

    def done(self, h):
        return self.clock() >= h["ready"]

    def collect(self, job, h):
        if self.overflow_once:
            self.overflow_once = False
            job.capacity *= 4
            return False
        for r in job.requests:
            r.pairs = int(self.ppp * r.cam.width * r.cam.height)
            r.image = ("img", r.rid)
        return True


@dataclasses.dataclass
class FakeScene:
    n: int


def _server(budget, max_views=4, slots=2, policy="fifo", **kw):
    clock = Clock()
    ex = FakeExec(clock, **kw)
    srv = S.Server({0: FakeScene(1000), 1: FakeScene(50_000)}, None, budget,
                   max_views=max_views, slots=slots, executor=ex, clock=clock, policy=policy)
    return srv, ex, clock


def test_batches_respect_view_limit_and_fifo():
    srv, ex, clock = _server(budget=10**9, max_views=3, slots=1)
    for k in range(7):
        srv.submit(0, Cam(64, 64))
    srv.poll()
    assert ex.launched == [[0, 1, 2]]
    clock.t = 1.0
    srv.poll()
    assert ex.launched[-1] == [3, 4, 5]
    clock.t = 2.0
    srv.poll()
    clock.t = 3.0
    srv.poll()
    assert ex.launched[-1] == [6]
    assert [r.rid for r in srv.done] == list(range(7))
    assert srv.idle()


def test_memory_budget_admission_and_release():
    srv, ex, clock = _server(budget=10**9, max_views=8, slots=2)
    one = srv.sched.request_bytes(S.Request(0, 1, Cam(512, 512), 0.0))
    srv, ex, clock = _server(budget=int(2.5 * one), max_views=8, slots=2)
    # two requests fit, the third waits
    for _ in range(3):
        srv.submit(1, Cam(512, 512))
    srv.poll()
    assert ex.launched == [[0, 1]]
    assert srv.sched.used == 2 * one and len(srv.sched.queue) == 1
    clock.t = 1.0
    srv.poll()                                  # frees memory, admits the third
    # the estimator has learned the real pair rate meanwhile
    assert ex.launched[-1] == [2] and srv.sched.used == srv.sched.in_flight[0].bytes < one
    clock.t = 2.0
    srv.poll()
    assert srv.idle() and srv.sched.used == 0


def test_request_larger_than_budget_is_rejected():
    srv, ex, clock = _server(budget=10**6)
    srv.submit(1, Cam(1920, 1080))
    assert len(srv.sched.rejected) == 1 and srv.idle()


def test_continuous_admission_into_free_slot():
    srv, ex, clock = _server(budget=10**9, max_views=8, slots=2)
    srv.submit(0, Cam(64, 64))
    srv.poll()
    clock.t = 0.001                             # first batch still in flight
    srv.submit(0, Cam(128, 64))
    srv.submit(1, Cam(32, 32))
    srv.poll()
    assert ex.launched == [[0], [1, 2]]         # joined the second slot at once
    assert [j.slot for j in srv.sched.in_flight] == [0, 1]
    clock.t = 0.1
    srv.poll()
    assert len(srv.done) == 3
    st = S.latency_stats(srv.done)
    assert st["n"] == 3 and st["p99_ms"] >= st["p50_ms"] > 0


def test_capacity_overflow_reruns_job():
    srv, ex, clock = _server(budget=10**9, overflow_once=True)
    srv.submit(0, Cam(64, 64))
    srv.poll()
    clock.t = 1.0
    srv.poll()                                  # overflow: relaunched
    assert len(ex.launched) == 2 and not srv.done
    clock.t = 2.0
    srv.poll()
    assert len(srv.done) == 1


def test_pair_estimator_learns_upwards():
    est = S.PairEstimator(prior_per_pixel=1.0, margin=1.0)
    a = est.estimate(3, 1000)
    est.update(3, 1000, 50_000)
    assert est.estimate(3, 1000) > a
    est.update(3, 1000, 10_000)                 # does not drop below the mean
    assert est.estimate(3, 1000) >= 30 * 1000


def test_replay_drives_arrivals():
    srv, ex, clock = _server(budget=10**9, max_views=4, slots=2, latency=0.002)
    arrivals = [(0.001 * k, k % 2, Cam(64, 64)) for k in range(20)]

    # advance the simulated clock inside the polling loop
    orig = srv.poll

    def poll():
        clock.t += 0.0005
        return orig()
    srv.poll = poll
    S.replay(srv, arrivals, spin=0)
    assert len(srv.done) == 20
    assert all(r.t_done >= r.t_arrival for r in srv.done)


def test_pool_first_fit_alignment_and_coalescing():
    p = S.Pool(10 * S.ALIGN + 17)
    assert p.size == 10 * S.ALIGN and p.largest_free() == p.size
    a = p.alloc(1)
    b = p.alloc(3 * S.ALIGN - 5)
    c = p.alloc(2 * S.ALIGN)
    assert (a, b, c) == (0, S.ALIGN, 4 * S.ALIGN)
    assert p.used == 6 * S.ALIGN and p.largest_free() == 4 * S.ALIGN
    assert p.alloc(5 * S.ALIGN) is None
    p.release(b)                       # hole of 3 blocks between a and c
    assert p.alloc(3 * S.ALIGN) == S.ALIGN
    p.release(S.ALIGN)
    p.release(a)
    p.release(c)                       # everything coalesces back
    assert p.free == [[0, p.size]] and p.used == 0


def test_size_class_batches_equal_resolutions_first():
    srv, ex, clock = _server(budget=10**10, max_views=4, slots=1, policy="size_class")
    sizes = [(512, 512), (1920, 1080), (512, 512), (1920, 1080), (512, 512)]
    for w, h in sizes:
        srv.submit(0, Cam(w, h))
    srv.poll()
    assert ex.launched == [[0, 2, 4]]   # the head's class, skipping the others
    clock.t = 1.0
    srv.poll()
    assert ex.launched[-1] == [1, 3]
    clock.t = 2.0
    srv.poll()
    assert srv.idle() and len(srv.done) == 5


def test_rerun_larger_than_the_pool_is_rejected():
    srv, ex, clock = _server(budget=10**9, overflow_once=True)
    one = srv.sched.request_bytes(S.Request(0, 0, Cam(64, 64), 0.0))
    srv, ex, clock = _server(budget=2 * one, overflow_once=True)
    ex_collect = ex.collect

    def collect(job, h):    # the pair list needs far more than the pool
        ok = ex_collect(job, h)
        if not ok:
            job.capacity = 10**9
        return ok
    ex.collect = collect
    r = srv.submit(0, Cam(64, 64))
    srv.poll()
    clock.t = 1.0
    srv.poll()
    assert r.failed and r in srv.sched.rejected and srv.idle() and srv.sched.used == 0


@pytest.mark.parametrize("policy", ["fifo", "size_class"])
def test_pool_never_overcommitted(policy):
    # random arrivals, sizes, scenes and latencies; overflows now and then:
    # after every poll the live blocks are disjoint and within the budget
    rng = np.random.default_rng(11)
    srv, ex, clock = _server(budget=60 << 20, max_views=6, slots=3, policy=policy)
    res = [(512, 512), (1280, 720), (1920, 1080), (64, 64)]
    for step in range(400):
        for _ in range(rng.poisson(0.8)):
            w, h = res[rng.integers(0, len(res))]
            srv.submit(int(rng.integers(0, 2)), Cam(w, h))
        if rng.uniform() < 0.05:
            ex.overflow_once = True
        ex.latency = float(rng.uniform(0.001, 0.01))
        clock.t += 0.002
        srv.poll()
        p = srv.sched.pool
        blocks = sorted(p.live.items())
        assert all(o1 + n1 <= o2 for (o1, n1), (o2, _) in zip(blocks, blocks[1:]))
        assert p.used <= p.size <= 60 << 20
        assert p.used == sum(j.bytes for j in srv.sched.in_flight)
    while not srv.idle():
        clock.t += 0.01
        srv.poll()
    assert srv.sched.used == 0 and len(srv.done) + len(srv.sched.rejected) == srv._rid
