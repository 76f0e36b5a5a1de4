#!/usr/bin/env python3
"""Benchmark of the local 3-D FFT hot path on one MI355X.

One step is one forward 512^3 complex-to-complex FP32 transform (z-, y- and
x-pass, Algorithm 1 of the AccFFT paper at P0 = P1 = 1) of a seeded
U[-1,1) complex64 grid already resident in HBM, out of place.  The JSON line
reports the whole transform's algorithmic HBM throughput (3 passes x one
read + one write of 8 bytes per element = 48 N bytes), the time per
transform, the dominant kernel's roofline (its algorithmic bytes over its
mean duration, from HIP events recorded around every pass during the timed
steps) and the FP64 CPU oracle timed on the host cores as a reported
baseline.

    python bench.py [--steps K] [--warmup W] [--no-cpu-baseline]
    python bench.py --mode copy    # plain 1 GiB device copy, for counter scaling
"""
from __future__ import annotations

import argparse
import hashlib
import json
import math
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

PEAK_HBM_GBS = 8000.0  # MI355X HBM3E, AMD published peak
N0 = N1 = N2 = 512


def csrc_hash() -> str:
    h = hashlib.sha256()
    d = os.path.join(ROOT, "paper_1506_07933_amd", "csrc")
    for name in sorted(os.listdir(d)):
        if name.endswith((".hip", ".hpp", ".inc")):
            with open(os.path.join(d, name), "rb") as f:
                h.update(name.encode())
                h.update(f.read())
    return h.hexdigest()[:16]


def load_traffic(kernel: str, launch_bytes: float):
    """Counter-measured HBM bytes per launch of `kernel`, if the committed
    counter summary was taken on the current kernel sources."""
    path = os.path.join(ROOT, "profiles", "traffic.json")
    if not os.path.exists(path):
        return None
    with open(path) as f:
        t = json.load(f)
    if t.get("csrc_hash") != csrc_hash():
        return None
    k = t.get("kernels", {}).get(kernel)
    if not k:
        return None
    return k.get("hbm_bytes_per_launch")


def copy_mode(args):
    import torch
    n = 1 << 27  # 1 GiB of complex64-sized elements as float64
    a = torch.empty(n, dtype=torch.float64, device="cuda").uniform_()
    b = torch.empty_like(a)
    for _ in range(args.warmup):
        b.copy_(a)
    torch.cuda.synchronize()
    s, e = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    s.record()
    for _ in range(args.steps):
        b.copy_(a)
    e.record()
    torch.cuda.synchronize()
    ms = s.elapsed_time(e) / args.steps
    print(json.dumps({"mode": "copy", "bytes_read": 8 * n, "bytes_written": 8 * n,
                      "ms": ms, "GBps": 16 * n / ms / 1e6}), flush=True)


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--mode", choices=["fft", "copy"], default="fft")
    args = ap.parse_args()
    world = int(os.environ.get("WORLD_SIZE", "1"))
    if args.gpus != 1 or world != 1:
        print("bench.py measures one GPU: the local FFT phases run on a single MI355X and this "
              "build has no multi-GPU exchange; run it with --gpus 1", file=sys.stderr)
        sys.exit(2)
    if args.mode == "copy":
        return copy_mode(args)

    import numpy as np
    import torch

    from paper_1506_07933_amd import Plan, synth
    from paper_1506_07933_amd.fft import profile_begin, profile_end

    n = N0 * N1 * N2
    x_host = synth.uniform_complex((N0, N1, N2), np.complex64, seed=0)
    x = torch.from_numpy(x_host).to("cuda:0")
    y = torch.empty_like(x)
    plan = Plan((N0, N1, N2), "c2c", "fp32")
    passes = [l for l in plan.describe().splitlines() if l.startswith("forward")]

    for _ in range(args.warmup):
        plan.forward(x, out=y)
    torch.cuda.synchronize()
    profile_begin(plan.handle, args.steps)
    start = torch.cuda.Event(enable_timing=True)
    stop = torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    start.record()
    for _ in range(args.steps):
        plan.forward(x, out=y)
    stop.record()
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    pass_ms, ncalls = profile_end(plan.handle)
    ms = start.elapsed_time(stop) / args.steps

    total_bytes = 3 * 16 * n  # 48 N: each pass reads and writes every complex64 once
    value = total_bytes / (ms * 1e-3) / 1e9
    names = ["z_contig", "y_strided", "x_strided"]
    dom = int(np.argmax(pass_ms))
    kbytes = 16 * n  # one pass: read + write of N complex64
    achieved = kbytes / (pass_ms[dom] * 1e-3) / 1e9
    kname = {0: "k_contig", 1: "k_strided(y)", 2: "k_strided(x)"}[dom]
    traffic = load_traffic(names[dom], kbytes)
    out = {
        "metric": "3-D FFT time & HBM GB/s vs peak (512^3 C2C fp32)",
        "value": round(value, 2),
        "unit": "GB/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(ms, 5),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": "c2c_forward_512x512x512_complex64", "grid": [N0, N1, N2],
                   "kind": "c2c", "precision": "fp32", "input": "re, im ~ U[-1,1), seed 0",
                   "placement": "out of place, input resident in HBM"},
        "gflops_5nlog2n": round(5 * n * math.log2(n) / (ms * 1e-3) / 1e9, 1),
        "frac_of_hbm_peak": round(value / PEAK_HBM_GBS, 4),
        "wall_ms_per_step": round(wall * 1e3 / args.steps, 5),
        "passes": [{"pass": names[i], "ms": round(pass_ms[i], 5),
                    "alg_GBps": round(kbytes / (pass_ms[i] * 1e-3) / 1e9, 1)}
                   for i in range(len(pass_ms))],
        "plan": passes,
        "roofline": {"bound": "hbm", "kernel": kname + " " + names[dom],
                     "achieved": round(achieved, 1), "peak": PEAK_HBM_GBS, "unit": "GB/s",
                     "frac": round(achieved / PEAK_HBM_GBS, 4), "traffic": traffic,
                     "alg_bytes_per_launch": kbytes, "launches_timed": ncalls},
    }
    if not args.no_cpu_baseline:
        import oracle
        x64 = x_host.astype(np.complex128)
        t0 = time.perf_counter()
        ref = oracle.fft3d_c2c(x64, -1)
        t_cpu = time.perf_counter() - t0
        got = y.cpu().numpy().astype(np.complex128)
        rel = float(np.linalg.norm(got - ref) / np.linalg.norm(ref))
        out["cpu_baseline"] = {"value": round(total_bytes / t_cpu / 1e9, 3), "unit": "GB/s",
                               "cores": oracle.max_threads(), "kind": "oracle",
                               "sample": "one full 512^3 forward transform of the same input, "
                                         "FP64, %.1f s" % t_cpu}
        out["rel_l2_vs_oracle"] = rel
    plan.close()
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
