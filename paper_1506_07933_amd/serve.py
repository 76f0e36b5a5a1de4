"""Continuous-batching server for spectral Poisson solves on one GPU.

Requests arrive open-loop (a pre-drawn arrival schedule replayed against the
clock).  Each request is one periodic Poisson solve lap(u) = f on an n^3 grid
(R2C forward, multiply by -1/|k|^2 with k = 0 zeroed, C2R inverse; the
"fast spectral operators" of the AccFFT paper, Sec. 1) in FP32 or FP64.

Scheduling (SchedulerCore, pure host logic):
  * arrived requests wait in a FIFO queue;
  * the HBM budget is one device pool of exactly that many bytes, allocated
    once; the head of the queue is admitted as soon as a slot is free and
    its device bytes (right-hand side + output + workspace) can be carved
    out of the pool (PoolAllocator: first fit, 256-byte aligned, freed
    ranges coalesce), so the budget bounds the memory requests really hold;
    a request larger than the whole pool is rejected at once with an error
    record instead of blocking the queue;
  * admitted requests are enqueued on their slot's stream, so work of
    different requests overlaps on the device; completions are polled and
    return their slot and pool range immediately, which is what lets
    requests that arrive while others run join the device work (continuous
    batching);
  * an executor failure fails only that request.
Latency = completion time - scheduled arrival time.

GpuPoissonExecutor keeps one plan per (n, precision) resident (twiddles on the
device), one stream per slot and the pool.  Each request draws its own
right-hand side on its slot's stream into its pool range (the Poisson recipe:
8 random Fourier modes plus N(0, 0.01) noise, seeded per request), then
solves; serving allocates nothing.  Every (n, precision) is run once at
start-up so no request pays for loading kernels.
"""
from __future__ import annotations

import collections
import dataclasses
import gc
import json
import math
import time
from typing import Callable, Dict, List, Optional, Sequence


@dataclasses.dataclass
class Request:
    rid: int
    t_arrival: float
    n: int
    prec: str
    variant: int = 0


@dataclasses.dataclass
class Record:
    rid: int
    n: int
    prec: str
    t_arrival: float
    t_admit: float = math.nan
    t_done: float = math.nan
    status: str = "pending"   # ok | rejected | failed
    error: str = ""
    slot: int = -1
    nbytes: int = 0

    @property
    def latency(self) -> float:
        return self.t_done - self.t_arrival


class PoolAllocator:
    """First-fit sub-allocation of one buffer of `size` bytes (offsets only;
    the executor owns the memory).  Ranges are rounded up to `align` bytes;
    a freed range is merged with free neighbours, so the pool never holds
    two adjacent free ranges."""

    def __init__(self, size: int, align: int = 256):
        if size < 1 or align < 1:
            raise ValueError("pool size and alignment must be positive")
        self.size = int(size) // align * align
        self.align = int(align)
        self.free: List[List[int]] = [[0, self.size]] if self.size else []
        self.used = 0

    def _round(self, nbytes: int) -> int:
        return max(1, -(-int(nbytes) // self.align)) * self.align

    def alloc(self, nbytes: int) -> Optional[int]:
        n = self._round(nbytes)
        for i, (off, ln) in enumerate(self.free):
            if ln >= n:
                if ln == n:
                    del self.free[i]
                else:
                    self.free[i] = [off + n, ln - n]
                self.used += n
                return off
        return None

    def release(self, off: int, nbytes: int) -> None:
        n = self._round(nbytes)
        i = 0
        while i < len(self.free) and self.free[i][0] < off:
            i += 1
        if (i > 0 and self.free[i - 1][0] + self.free[i - 1][1] > off) or \
                (i < len(self.free) and off + n > self.free[i][0]) or off < 0 or off + n > self.size:
            raise ValueError("release of [%d, %d) overlaps free memory" % (off, off + n))
        self.free.insert(i, [off, n])
        if i + 1 < len(self.free) and off + n == self.free[i + 1][0]:
            self.free[i][1] += self.free[i + 1][1]
            del self.free[i + 1]
        if i > 0 and self.free[i - 1][0] + self.free[i - 1][1] == off:
            self.free[i - 1][1] += self.free[i][1]
            del self.free[i]
        self.used -= n

    def fits(self, nbytes: int) -> bool:
        return self._round(nbytes) <= self.size


class SchedulerCore:
    """FIFO admission by slots and a pool of `budget_bytes`; executor-agnostic.

    executor must provide:
      bytes_needed(req) -> int
      submit(req, slot, offset) -> handle  (enqueue device work using the pool
                                           range at `offset`; may raise)
      poll(handle) -> bool                 (True once the work has completed; may raise)
      release(handle)                      (called before the range returns to the pool)
    """

    def __init__(self, executor, budget_bytes: int, slots: int):
        if slots < 1 or budget_bytes < 1:
            raise ValueError("need at least one slot and a positive budget")
        self.ex = executor
        self.pool = PoolAllocator(int(budget_bytes))
        self.budget = self.pool.size
        self.free_slots = list(range(slots))[::-1]
        self.queue: collections.deque = collections.deque()
        self.inflight: Dict[int, tuple] = {}
        self.bytes_in_flight = 0
        self.peak_bytes = 0
        self.records: Dict[int, Record] = {}
        self.depth_log: List[tuple] = []

    def arrive(self, req: Request, now: float) -> None:
        self.records[req.rid] = Record(req.rid, req.n, req.prec, req.t_arrival)
        self.queue.append(req)

    def _finish(self, rid: int, now: float, status: str, err: str = "") -> None:
        rec = self.records[rid]
        rec.t_done = now
        rec.status = status
        rec.error = err

    def step(self, now: float) -> int:
        """Poll completions, then admit from the queue.  Returns the number
        of state changes (0 means the caller may idle briefly)."""
        changes = 0
        for rid in list(self.inflight):
            handle, slot, nbytes, off = self.inflight[rid]
            try:
                finished = self.ex.poll(handle)
                err = ""
            except Exception as e:  # noqa: BLE001 - isolate the failing request
                finished, err = True, repr(e)
            if finished:
                del self.inflight[rid]
                self.ex.release(handle)
                self.pool.release(off, nbytes)
                self.bytes_in_flight -= nbytes
                self.free_slots.append(slot)
                self._finish(rid, now, "failed" if err else "ok", err)
                changes += 1
        while self.queue and self.free_slots:
            req = self.queue[0]
            need = int(self.ex.bytes_needed(req))
            if not self.pool.fits(need):
                self.queue.popleft()
                self._finish(req.rid, now, "rejected", "needs %d bytes, budget %d" % (need, self.budget))
                changes += 1
                continue
            off = self.pool.alloc(need)
            if off is None:
                break  # FIFO: the head waits for memory, nothing overtakes it
            self.queue.popleft()
            slot = self.free_slots.pop()
            rec = self.records[req.rid]
            rec.t_admit, rec.slot, rec.nbytes = now, slot, need
            try:
                handle = self.ex.submit(req, slot, off)
            except Exception as e:  # noqa: BLE001
                self.free_slots.append(slot)
                self.pool.release(off, need)
                self._finish(req.rid, now, "failed", repr(e))
                changes += 1
                continue
            self.inflight[req.rid] = (handle, slot, need, off)
            self.bytes_in_flight += need
            self.peak_bytes = max(self.peak_bytes, self.bytes_in_flight)
            changes += 1
        state = (len(self.queue), len(self.inflight), self.bytes_in_flight)
        if not self.depth_log or self.depth_log[-1][1:] != state:
            self.depth_log.append((now,) + state)
        return changes

    @property
    def idle(self) -> bool:
        return not self.queue and not self.inflight


def run_open_loop(schedule: Sequence[Request], core: SchedulerCore,
                  clock: Callable[[], float], idle: Optional[Callable[[], None]] = None,
                  max_wall: float = 600.0) -> Dict[int, Record]:
    """Replay the arrival schedule (times relative to the first clock read)
    against `clock`, stepping the scheduler until every request finished."""
    t0 = clock()
    pending = collections.deque(sorted(schedule, key=lambda r: r.t_arrival))
    while pending or not core.idle:
        now = clock() - t0
        if now > max_wall:
            raise TimeoutError("serving replay exceeded %.0f s" % max_wall)
        while pending and pending[0].t_arrival <= now:
            core.arrive(pending.popleft(), now)
        if core.step(now) == 0 and idle is not None:
            idle()
    return core.records


def _pct(sorted_vals, p):
    """The p-th percentile (nearest rank) of an ascending list."""
    if not sorted_vals:
        return math.nan
    k = min(len(sorted_vals) - 1, max(0, int(math.ceil(p / 100.0 * len(sorted_vals))) - 1))
    return sorted_vals[k]


def summarize(records: Dict[int, Record], wall: float, bytes_per_req: Callable[[Record], float]):
    ok = [r for r in records.values() if r.status == "ok"]
    lat = sorted(r.latency for r in ok)

    def pct(p):
        if not lat:
            return math.nan
        k = min(len(lat) - 1, max(0, int(math.ceil(p / 100.0 * len(lat))) - 1))
        return lat[k]

    span = (max(r.t_done for r in ok) - min(r.t_arrival for r in ok)) if ok else math.nan
    moved = sum(bytes_per_req(r) for r in ok)
    return {
        "requests": len(records), "ok": len(ok),
        "rejected": sum(r.status == "rejected" for r in records.values()),
        "failed": sum(r.status == "failed" for r in records.values()),
        "p50_ms": pct(50) * 1e3, "p99_ms": pct(99) * 1e3, "mean_ms": (sum(lat) / len(lat) * 1e3) if lat else math.nan,
        "throughput_req_s": len(ok) / span if span and span > 0 else math.nan,
        "throughput_GBps": moved / span / 1e9 if span and span > 0 else math.nan,
        "wall_s": wall,
    }


# ------------------------------------------------------------ GPU executor

def poisson_alg_bytes(n: int, prec: str) -> float:
    """Algorithmic HBM bytes of one solve: R2C (read n^3 reals, write the half
    spectrum), y and x passes (read + write the half spectrum each), the
    multiply (read + write), and the mirror-image inverse."""
    esz = 4 if prec == "fp32" else 8
    real = n ** 3 * esz
    half = n * n * (n // 2 + 1) * 2 * esz
    fwd = (real + half) + 2 * (2 * half)
    return 2 * fwd + 2 * half


class GpuPoissonExecutor:
    """Device side of the server: resident plans, one stream per slot and the
    budget pool.  A request's pool range holds [f | u | ws]: its right-hand
    side (drawn on the device), its solution and the Poisson workspace."""

    ALIGN = 256

    def __init__(self, sizes: Sequence[int], precs: Sequence[str], slots: int, budget_bytes: int,
                 seed: int = 0, device: str = "cuda:0"):
        import torch

        from .fft import Plan
        self.torch = torch
        self.device = device
        self.seed = seed
        self.plans: Dict[tuple, Plan] = {}
        self.streams = [torch.cuda.Stream(device=device) for _ in range(slots)]
        for n in sizes:
            for prec in precs:
                self.plans[(n, prec)] = Plan((n, n, n), "r2c", prec)
        # the budget: one pool, allocated once (sub-ranges per request)
        self.pool = torch.empty(int(budget_bytes) // self.ALIGN * self.ALIGN, dtype=torch.uint8, device=device)
        nmax = max(sizes)
        # per-slot pinned staging of the generator's per-axis factors (a slot's
        # next request starts only after its previous one has completed)
        self.staging = [torch.empty(3 * 8 * nmax, dtype=torch.complex128, pin_memory=True) for _ in range(slots)]
        # per slot: events around the solve itself (after the right-hand side
        # is drawn), for the device time of each solve
        self.events = [torch.cuda.Event(enable_timing=True) for _ in range(slots)]
        self.events0 = [torch.cuda.Event(enable_timing=True) for _ in range(slots)]
        self.solve_ms: Dict[int, float] = {}
        self.outputs: Dict[int, object] = {}
        self.inputs: Dict[int, object] = {}
        self.keep_outputs = False
        # warm-up: every plan and right-hand-side shape once (kernels and the
        # generator's library routines load on first use), and one solve and
        # one event on every slot's stream (the first use of a stream sets it
        # up, which took tens of milliseconds)
        for (n, prec), p in sorted(self.plans.items(), key=lambda kv: kv[0][0]):
            if self.bytes_for(n, prec) > self.pool.numel():
                continue
            f, u, ws = self._views(0, n, prec)
            self._draw(f, 0, self.streams[0], 0)
            p.poisson(f, out=u, ws=ws, stream=self.streams[0])
            torch.cuda.synchronize()
        small = min(k for k in self.plans if self.bytes_for(*k) <= self.pool.numel())
        for slot, s in enumerate(self.streams):
            f, u, ws = self._views(0, *small)
            self._draw(f, 0, s, slot)
            self.plans[small].poisson(f, out=u, ws=ws, stream=s)
            self.events[slot].record(s)
            self.events[slot].query()
            torch.cuda.synchronize()

    def _rnd(self, b: int) -> int:
        return -(-b // self.ALIGN) * self.ALIGN

    def bytes_for(self, n: int, prec: str) -> int:
        esz = 4 if prec == "fp32" else 8
        return 2 * self._rnd(n ** 3 * esz) + self._rnd(self.plans[(n, prec)].poisson_ws_bytes)

    def _views(self, off: int, n: int, prec: str):
        torch = self.torch
        esz = 4 if prec == "fp32" else 8
        fb = self._rnd(n ** 3 * esz)
        dt = torch.float32 if prec == "fp32" else torch.float64
        a = self.pool
        f = a[off:off + n ** 3 * esz].view(dt).view(n, n, n)
        u = a[off + fb:off + fb + n ** 3 * esz].view(dt).view(n, n, n)
        ws = a[off + 2 * fb:off + 2 * fb + self.plans[(n, prec)].poisson_ws_bytes]
        return f, u, ws

    def _draw(self, f, rid: int, stream, slot: int) -> None:
        from . import synth
        synth.poisson_rhs_device(f, self.rhs_seed(rid), stream=stream, staging=self.staging[slot])

    def rhs_seed(self, rid: int) -> int:
        return self.seed * 1000003 + rid

    def bytes_needed(self, req: Request) -> int:
        return self.bytes_for(req.n, req.prec)

    def submit(self, req: Request, slot: int, offset: int):
        p = self.plans[(req.n, req.prec)]
        s = self.streams[slot]
        f, u, ws = self._views(offset, req.n, req.prec)
        self._draw(f, req.rid, s, slot)
        ev0 = self.events0[slot]
        ev0.record(s)
        p.poisson(f, out=u, ws=ws, stream=s)
        ev = self.events[slot]
        ev.record(s)
        return (req, ev, f, u, slot, ev0)

    def poll(self, handle) -> bool:
        return handle[1].query()

    def release(self, handle) -> None:
        req, ev, f, u, slot, ev0 = handle
        self.solve_ms[req.rid] = ev0.elapsed_time(ev)
        if self.keep_outputs:
            # copies for the caller (tests), finished before the pool range
            # is handed to the next request
            s = self.streams[slot]
            with self.torch.cuda.stream(s):
                self.outputs[req.rid] = u.clone()
                self.inputs[req.rid] = f.clone()
            s.synchronize()

    def run_alone(self, req: Request):
        """The same request on an otherwise idle device (offset 0 of the
        pool, slot 0); returns copies of (f, u)."""
        self.torch.cuda.synchronize()
        h = self.submit(req, 0, 0)
        h[1].synchronize()
        out = (h[2].clone(), h[3].clone())
        self.torch.cuda.synchronize()
        return out

    def close(self):
        for p in self.plans.values():
            p.close()


def timeline(depth_log, points: int = 24):
    """The scheduler's state over the replay, resampled at `points` equal
    steps: (t_s, queue depth, requests in flight, bytes in flight)."""
    if not depth_log:
        return []
    t_end = depth_log[-1][0]
    out, k = [], 0
    for i in range(points):
        t = t_end * i / max(1, points - 1)
        while k + 1 < len(depth_log) and depth_log[k + 1][0] <= t:
            k += 1
        out.append((round(t, 4),) + tuple(depth_log[k][1:]))
    return out


def mean_queue_depth(depth_log) -> float:
    """Time-weighted mean number of waiting requests."""
    if len(depth_log) < 2:
        return 0.0
    area = sum((depth_log[i + 1][0] - depth_log[i][0]) * depth_log[i][1] for i in range(len(depth_log) - 1))
    span = depth_log[-1][0] - depth_log[0][0]
    return area / span if span > 0 else 0.0


def serve(n_requests: int = 2000, rate: float = 200.0, seed: int = 0, sizes=(64, 128, 256, 384, 512),
          slots: int = 4, budget_gb: float = 16.0, keep_outputs: bool = False, schedule=None):
    """Run the open-loop Poisson-solve workload on the GPU; returns
    (summary, records, executor).  `schedule` (a list of (t, n, prec))
    replaces the drawn arrival schedule when given."""
    import torch

    from . import synth
    sched = schedule if schedule is not None else synth.arrival_schedule(n_requests, rate, seed=seed, sizes=sizes)
    reqs = [Request(i, t, n, prec, variant=i) for i, (t, n, prec) in enumerate(sched)]
    precs = sorted({r.prec for r in reqs})
    budget = int(budget_gb * 2 ** 30)
    ex = GpuPoissonExecutor(sorted({r.n for r in reqs}), precs, slots, budget, seed=seed)
    ex.keep_outputs = keep_outputs
    core = SchedulerCore(ex, budget, slots)
    # The replay must not pause for the garbage collector: a full collection
    # over the interpreter's objects (torch's included) took ~33 ms and landed
    # on the first requests.  Collect once, move everything alive to the
    # permanent generation, and keep automatic collection off while serving.
    gc.collect()
    gc.freeze()
    gc_was_enabled = gc.isenabled()
    gc.disable()
    try:
        t0 = time.perf_counter()
        recs = run_open_loop(reqs, core, time.perf_counter)
        torch.cuda.synchronize()
        wall = time.perf_counter() - t0
    finally:
        if gc_was_enabled:
            gc.enable()
        gc.unfreeze()
    summary = summarize(recs, wall, lambda r: poisson_alg_bytes(r.n, r.prec))
    waited = [r.t_admit - r.t_arrival for r in recs.values() if r.status == "ok"]
    summary.update({"slots": slots, "budget_GB": budget_gb, "rate_req_s": rate if schedule is None else None,
                    "peak_bytes_in_flight": core.peak_bytes,
                    "max_queue_depth": max(d[1] for d in core.depth_log) if core.depth_log else 0,
                    "mean_queue_depth": mean_queue_depth(core.depth_log),
                    "queued_requests": sum(1 for w in waited if w > 1e-3),
                    "max_admission_wait_ms": max(waited) * 1e3 if waited else math.nan,
                    # device time of the solves alone (events around each solve, after its
                    # right-hand side is drawn); p50_ms / p99_ms include the draw and any wait
                    "p50_solve_ms": _pct(sorted(ex.solve_ms.values()), 50),
                    "p99_solve_ms": _pct(sorted(ex.solve_ms.values()), 99),
                    "timeline_t_queue_inflight_bytes": timeline(core.depth_log)})
    return summary, recs, ex


if __name__ == "__main__":
    import argparse
    ap = argparse.ArgumentParser()
    ap.add_argument("--requests", type=int, default=2000)
    ap.add_argument("--rate", type=float, default=200.0)
    ap.add_argument("--slots", type=int, default=4)
    ap.add_argument("--budget-gb", type=float, default=16.0)
    ap.add_argument("--seed", type=int, default=0)
    a = ap.parse_args()
    s, _, ex = serve(a.requests, a.rate, a.seed, slots=a.slots, budget_gb=a.budget_gb)
    print(json.dumps(s))
    ex.close()
