"""Serving scheduler on the CPU: a fake executor and a virtual clock drive
SchedulerCore through the open-loop replay.  Checks the admission rules the
GPU server relies on: the HBM budget and slot count are never exceeded,
admission is FIFO, a request that can never fit is rejected instead of
blocking the queue, and an executor failure fails only its own request."""
import pytest

from paper_1506_07933_amd.serve import (PoolAllocator, Request, SchedulerCore, mean_queue_depth,
                                        run_open_loop, summarize, timeline)


class Clock:
    def __init__(self):
        self.t = 0.0

    def __call__(self):
        return self.t

    def tick(self, dt=1e-4):
        self.t += dt


class FakeExec:
    """bytes = n (arbitrary units); duration = n * 1e-5 s of virtual time."""

    def __init__(self, clock, fail_submit=(), fail_poll=(), pool_size=1 << 40):
        self.clock = clock
        self.pool_size = pool_size
        self.ranges = {}
        self.fail_submit = set(fail_submit)
        self.fail_poll = set(fail_poll)
        self.admitted = []
        self.max_concurrent = 0
        self.live = 0

    def bytes_needed(self, req):
        return req.n

    def submit(self, req, slot, offset):
        if req.rid in self.fail_submit:
            raise RuntimeError("injected submit failure")
        self.admitted.append(req.rid)
        self.live += 1
        self.max_concurrent = max(self.max_concurrent, self.live)
        # the ranges of requests in flight never overlap and stay in the pool
        for (o, n) in self.ranges.values():
            assert offset + req.n <= o or o + n <= offset
        assert 0 <= offset and offset + req.n <= self.pool_size
        self.ranges[req.rid] = (offset, req.n)
        return (req, self.clock() + req.n * 1e-5)

    def poll(self, h):
        req, t_end = h
        if req.rid in self.fail_poll and self.clock() >= t_end:
            raise RuntimeError("injected device failure")
        return self.clock() >= t_end

    def release(self, h):
        self.live -= 1
        del self.ranges[h[0].rid]


def make_requests(sizes, gap=1e-4):
    return [Request(i, i * gap, n, "fp32") for i, n in enumerate(sizes)]


def test_budget_slots_and_fifo():
    clock = Clock()
    ex = FakeExec(clock, pool_size=1024)
    core = SchedulerCore(ex, budget_bytes=1024, slots=3)
    sizes = [400, 300, 500, 100, 250, 600, 50, 700, 200, 350] * 5
    recs = run_open_loop(make_requests(sizes), core, clock, idle=clock.tick)
    assert all(r.status == "ok" for r in recs.values())
    assert core.peak_bytes <= 1024
    assert ex.max_concurrent <= 3
    assert max(d[1] for d in core.depth_log) > 0          # the budget made requests wait
    assert core.pool.used == 0 and core.pool.free == [[0, 1024]]
    assert ex.admitted == sorted(ex.admitted)  # FIFO
    for r in recs.values():
        assert r.t_done - r.t_admit >= r.n * 1e-5 - 1e-12
        assert r.latency >= r.t_done - r.t_admit
    s = summarize(recs, clock(), lambda r: r.n)
    assert s["ok"] == len(sizes) and s["p99_ms"] >= s["p50_ms"] > 0


def test_oversize_request_is_rejected_not_blocking():
    clock = Clock()
    ex = FakeExec(clock)
    core = SchedulerCore(ex, budget_bytes=512, slots=2)
    recs = run_open_loop(make_requests([100, 800, 200, 300]), core, clock, idle=clock.tick)
    assert recs[1].status == "rejected" and "budget" in recs[1].error
    assert [recs[i].status for i in (0, 2, 3)] == ["ok"] * 3


def test_failures_are_isolated():
    clock = Clock()
    ex = FakeExec(clock, fail_submit={2}, fail_poll={5})
    core = SchedulerCore(ex, budget_bytes=10000, slots=4)
    recs = run_open_loop(make_requests([100] * 10), core, clock, idle=clock.tick)
    assert recs[2].status == "failed" and "submit" in recs[2].error
    assert recs[5].status == "failed" and "device" in recs[5].error
    assert sum(r.status == "ok" for r in recs.values()) == 8
    assert core.bytes_in_flight == 0 and len(core.free_slots) == 4


def test_requests_arriving_during_work_join_it():
    """Continuous batching: a request arriving while another runs is admitted
    before the first completes when a slot and memory are free."""
    clock = Clock()
    ex = FakeExec(clock)
    core = SchedulerCore(ex, budget_bytes=10000, slots=4)
    reqs = [Request(0, 0.0, 1000, "fp32"), Request(1, 0.001, 100, "fp32")]
    recs = run_open_loop(reqs, core, clock, idle=clock.tick)
    assert recs[1].t_admit < recs[0].t_done
    assert recs[1].t_done < recs[0].t_done


def test_bad_configuration():
    with pytest.raises(ValueError):
        SchedulerCore(FakeExec(Clock()), budget_bytes=0, slots=1)
    with pytest.raises(ValueError):
        SchedulerCore(FakeExec(Clock()), budget_bytes=10, slots=0)


def test_pool_allocator_first_fit_and_coalescing():
    p = PoolAllocator(4096, align=256)
    a = p.alloc(100)      # 256
    b = p.alloc(600)      # 768
    c = p.alloc(1000)     # 1024
    assert (a, b, c) == (0, 256, 1024) and p.used == 2048
    assert p.alloc(2049) is None          # 2048 left
    p.release(b, 600)                     # hole [256, 1024)
    assert p.alloc(800) == 2048           # 1024 rounded: the 768-byte hole is too small
    assert p.alloc(700) == 256            # first fit reuses the hole
    p.release(2048, 800)
    p.release(256, 700)
    p.release(a, 100)                     # merges with the hole: [0, 1024)
    assert p.free[0] == [0, 1024]
    p.release(c, 1000)                    # everything free again, one range
    assert p.free == [[0, 4096]] and p.used == 0
    with pytest.raises(ValueError):
        p.release(0, 256)                 # double free
    assert not p.fits(4097) and p.fits(4096)


def test_fragmented_pool_makes_the_head_wait():
    """Admission needs a contiguous range: with 600 of 1024 bytes free in two
    holes, a 512-byte request waits (FIFO) until a neighbour completes."""
    clock = Clock()
    ex = FakeExec(clock, pool_size=1024)
    core = SchedulerCore(ex, budget_bytes=1024, slots=4)
    reqs = [Request(0, 0.0, 256, "fp32"), Request(1, 0.0, 256, "fp32"), Request(2, 0.0, 2000 // 8, "fp32"),
            Request(3, 0.0, 512, "fp32")]
    # durations n * 1e-5: request 3 must wait for request 0 or 1 to free a range
    recs = run_open_loop(reqs, core, clock, idle=clock.tick)
    assert all(r.status == "ok" for r in recs.values())
    assert recs[3].t_admit >= min(recs[0].t_done, recs[1].t_done)
    assert core.peak_bytes <= 1024
    tl = timeline(core.depth_log, points=5)
    assert len(tl) == 5 and tl[0][0] == 0.0
    assert mean_queue_depth(core.depth_log) > 0
