"""Continuous-batching server for spectral Poisson solves on one GPU.

Requests arrive open-loop (a pre-drawn arrival schedule replayed against the
clock).  Each request is one periodic Poisson solve lap(u) = f on an n^3 grid
(R2C forward, multiply by -1/|k|^2 with k = 0 zeroed, C2R inverse; the
"fast spectral operators" of the AccFFT paper, Sec. 1) in FP32 or FP64.

Scheduling (SchedulerCore, pure host logic):
  * arrived requests wait in a FIFO queue;
  * the head of the queue is admitted as soon as a slot is free and its
    device bytes (output + workspace) fit in the HBM budget on top of the
    bytes of the requests in flight; a request that could never fit is
    rejected at once with an error record instead of blocking the queue;
  * admitted requests are enqueued on their slot's stream, so work of
    different requests overlaps on the device; completions are polled and
    free their slot and bytes immediately, which is what lets requests that
    arrive while others run join the device work (continuous batching);
  * an executor failure fails only that request.
Latency = completion time - scheduled arrival time.

GpuPoissonExecutor keeps one plan per (n, precision) resident (twiddles on the
device), one stream per slot, a device-resident pool of right-hand sides, and
one preallocated arena per slot that holds the largest request's output and
workspace, so serving allocates nothing; every (n, precision) is run once at
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


class SchedulerCore:
    """FIFO admission by slots and HBM budget; executor-agnostic.

    executor must provide:
      bytes_needed(req) -> int
      submit(req, slot) -> handle       (enqueue device work; may raise)
      poll(handle) -> bool              (True once the work has completed; may raise)
      release(handle)                   (free the request's buffers)
    """

    def __init__(self, executor, budget_bytes: int, slots: int):
        if slots < 1 or budget_bytes < 1:
            raise ValueError("need at least one slot and a positive budget")
        self.ex = executor
        self.budget = int(budget_bytes)
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
            handle, slot, nbytes = self.inflight[rid]
            try:
                finished = self.ex.poll(handle)
                err = ""
            except Exception as e:  # noqa: BLE001 - isolate the failing request
                finished, err = True, repr(e)
            if finished:
                del self.inflight[rid]
                self.ex.release(handle)
                self.bytes_in_flight -= nbytes
                self.free_slots.append(slot)
                self._finish(rid, now, "failed" if err else "ok", err)
                changes += 1
        while self.queue and self.free_slots:
            req = self.queue[0]
            need = int(self.ex.bytes_needed(req))
            if need > self.budget:
                self.queue.popleft()
                self._finish(req.rid, now, "rejected", "needs %d bytes, budget %d" % (need, self.budget))
                changes += 1
                continue
            if self.bytes_in_flight + need > self.budget:
                break  # FIFO: the head waits for memory, nothing overtakes it
            self.queue.popleft()
            slot = self.free_slots.pop()
            rec = self.records[req.rid]
            rec.t_admit, rec.slot, rec.nbytes = now, slot, need
            try:
                handle = self.ex.submit(req, slot)
            except Exception as e:  # noqa: BLE001
                self.free_slots.append(slot)
                self._finish(req.rid, now, "failed", repr(e))
                changes += 1
                continue
            self.inflight[req.rid] = (handle, slot, need)
            self.bytes_in_flight += need
            self.peak_bytes = max(self.peak_bytes, self.bytes_in_flight)
            changes += 1
        self.depth_log.append((now, len(self.queue), len(self.inflight), self.bytes_in_flight))
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
    def __init__(self, sizes: Sequence[int], precs: Sequence[str], slots: int, variants: int = 2,
                 seed: int = 0, device: str = "cuda:0"):
        import torch

        from . import synth
        from .fft import Plan
        self.torch = torch
        self.device = device
        self.plans: Dict[tuple, Plan] = {}
        self.rhs: Dict[tuple, list] = {}
        self.streams = [torch.cuda.Stream(device=device) for _ in range(slots)]
        for n in sizes:
            for prec in precs:
                p = Plan((n, n, n), "r2c", prec)
                self.plans[(n, prec)] = p
                dt = torch.float32 if prec == "fp32" else torch.float64
                self.rhs[(n, prec)] = [synth.poisson_rhs_torch(n, seed * 1000 + 17 * n + v, dt, device)
                                       for v in range(variants)]
        # one arena per slot: output (256-byte aligned) + workspace of the largest request
        self.arena_bytes = max(self._layout(n, prec)[2] for (n, prec) in self.plans)
        self.arenas = [torch.empty(self.arena_bytes, dtype=torch.uint8, device=device) for _ in range(slots)]
        self.events = [torch.cuda.Event() for _ in range(slots)]
        # warm-up: every plan once, so kernels are loaded before serving
        # starts, and one solve and one event on every slot's stream (the
        # first use of a stream sets it up, which took tens of milliseconds)
        for (n, prec), p in self.plans.items():
            u, ws = self._views(0, n, prec)
            p.poisson(self.rhs[(n, prec)][0], out=u, ws=ws)
        n_min, p_min = min(self.plans.items(), key=lambda kv: kv[0][0] ** 3)
        for slot, s in enumerate(self.streams):
            u, ws = self._views(slot, *n_min)
            p_min.poisson(self.rhs[n_min][0], out=u, ws=ws, stream=s)
            self.events[slot].record(s)
            self.events[slot].query()
        torch.cuda.synchronize()
        self.outputs: Dict[int, object] = {}
        self.keep_outputs = False

    def _layout(self, n: int, prec: str):
        esz = 4 if prec == "fp32" else 8
        u_bytes = n ** 3 * esz
        ws_off = (u_bytes + 255) // 256 * 256
        return u_bytes, ws_off, ws_off + self.plans[(n, prec)].poisson_ws_bytes

    def _views(self, slot: int, n: int, prec: str):
        torch = self.torch
        u_bytes, ws_off, end = self._layout(n, prec)
        a = self.arenas[slot]
        dt = torch.float32 if prec == "fp32" else torch.float64
        return a[:u_bytes].view(dt).view(n, n, n), a[ws_off:end]

    def bytes_needed(self, req: Request) -> int:
        return self._layout(req.n, req.prec)[2]

    def submit(self, req: Request, slot: int):
        p = self.plans[(req.n, req.prec)]
        f = self.rhs[(req.n, req.prec)][req.variant % len(self.rhs[(req.n, req.prec)])]
        s = self.streams[slot]
        u, ws = self._views(slot, req.n, req.prec)
        p.poisson(f, out=u, ws=ws, stream=s)
        ev = self.events[slot]
        ev.record(s)
        return (req, ev, u, ws, slot)

    def poll(self, handle) -> bool:
        return handle[1].query()

    def release(self, handle) -> None:
        req, ev, u, ws, _ = handle
        if self.keep_outputs:
            # the slot's arena is reused by the next request: copy the output
            # on the slot's stream, ahead of that request's work
            with self.torch.cuda.stream(self.streams[handle[4]]):
                self.outputs[req.rid] = u.clone()

    def close(self):
        for p in self.plans.values():
            p.close()


def serve(n_requests: int = 2000, rate: float = 200.0, seed: int = 0, sizes=(64, 128, 256, 384, 512),
          slots: int = 4, budget_gb: float = 32.0, keep_outputs: bool = False):
    """Run the open-loop Poisson-solve workload on the GPU; returns
    (summary, records, executor)."""
    import torch

    from . import synth
    sched = synth.arrival_schedule(n_requests, rate, seed=seed, sizes=sizes)
    reqs = [Request(i, t, n, prec, variant=i) for i, (t, n, prec) in enumerate(sched)]
    precs = sorted({r.prec for r in reqs})
    ex = GpuPoissonExecutor(sorted({r.n for r in reqs}), precs, slots, seed=seed)
    ex.keep_outputs = keep_outputs
    core = SchedulerCore(ex, int(budget_gb * 2 ** 30), slots)
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
    summary.update({"slots": slots, "budget_GB": budget_gb, "rate_req_s": rate,
                    "peak_bytes_in_flight": core.peak_bytes,
                    "max_queue_depth": max(d[1] for d in core.depth_log) if core.depth_log else 0})
    return summary, recs, ex


if __name__ == "__main__":
    import argparse
    ap = argparse.ArgumentParser()
    ap.add_argument("--requests", type=int, default=2000)
    ap.add_argument("--rate", type=float, default=200.0)
    ap.add_argument("--slots", type=int, default=4)
    ap.add_argument("--budget-gb", type=float, default=32.0)
    ap.add_argument("--seed", type=int, default=0)
    a = ap.parse_args()
    s, _, ex = serve(a.requests, a.rate, a.seed, slots=a.slots, budget_gb=a.budget_gb)
    print(json.dumps(s))
    ex.close()
