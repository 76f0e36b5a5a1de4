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
    """Hash of the sources that make the single-transform kernels and their
    launch configurations (the batched executor's and the tuner's sources are
    left out: they do not change what the headline transform runs)."""
    h = hashlib.sha256()
    d = os.path.join(ROOT, "paper_1506_07933_amd", "csrc")
    for name in sorted(os.listdir(d)):
        if name.startswith(("batch", "tune")):
            continue
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


def slab_share(torch, np, time_fn, warmup, steps):
    """One task's share of the 512^3 C2C FP32 slab transform over 4 tasks
    (Algorithm 3): the 2-D FFTs of its 128 x-planes written in the send
    layout, and the x-FFT of a received 512 x 128 x 512 slab (the send buffer
    stands in for the receive buffer: one GPU moves no blocks); then the
    inverse stages.  Algorithmic bytes: one read and one write of the share
    per axis pass."""
    from paper_1506_07933_amd import SlabPlan, synth
    sp = SlabPlan((512, 512, 512), 4, "c2c", "fp32")
    cd = torch.complex64
    a = torch.from_numpy(synth.uniform_complex(sp.slab_shape, np.complex64, seed=0)).cuda()
    send = torch.empty(sp.send_shape, dtype=cd, device="cuda")
    recv = torch.empty(sp.send_shape, dtype=cd, device="cuda")
    mid = torch.empty(sp.mid_shape, dtype=cd, device="cuda")
    sh = torch.empty(sp.share_shape, dtype=cd, device="cuda")
    back = torch.empty(sp.slab_shape, dtype=cd, device="cuda")
    ns = a.numel()
    loc = time_fn(lambda: sp.forward_local(a, send, mid, fused=True), warmup, steps)
    xf = time_fn(lambda: sp.forward_x(send, sh), warmup, steps)
    unf = time_fn(lambda: sp.forward_local(a, send, mid, fused=False), warmup, max(3, steps // 4))
    recv.copy_(send)
    xi = time_fn(lambda: sp.inverse_x(sh, send), warmup, steps)
    li = time_fn(lambda: sp.inverse_local(recv, send, back, fused=True), warmup, steps)
    sp.close()
    fwd = loc + xf
    return {"forward_local_2d_ms": round(loc, 4), "forward_x_ms": round(xf, 4), "forward_ms": round(fwd, 4),
            "forward_alg_GBps": round(48 * ns / fwd / 1e6, 1),
            "forward_local_unfused_ms": round(unf, 4),
            "inverse_x_ms": round(xi, 4), "inverse_local_2d_ms": round(li, 4),
            "inverse_alg_GBps": round(48 * ns / (xi + li) / 1e6, 1)}


def nd_4d(torch, time_fn, warmup, steps):
    """The paper's 4-D C2C case, 512 x 256 x 128 x 64 complex64 (8 GiB), one
    forward and one inverse (in place) through the rank-4 plan; input
    U[-1,1) from torch's device generator seeded with 0.  Algorithmic bytes:
    one read and one write per axis pass, 4 x 16 bytes per element."""
    from paper_1506_07933_amd import Plan
    shape = (512, 256, 128, 64)
    g = torch.Generator(device="cuda")
    g.manual_seed(0)
    x = torch.complex(torch.rand(shape, device="cuda", generator=g) * 2 - 1,
                      torch.rand(shape, device="cuda", generator=g) * 2 - 1)
    y = torch.empty_like(x)
    p = Plan(shape, "c2c", "fp32")
    f = time_fn(lambda: p.forward(x, out=y), warmup, steps)
    i = time_fn(lambda: p.inverse(y, out=y), warmup, steps)
    p.close()
    n = x.numel()
    return {"forward_ms": round(f, 4), "forward_alg_GBps": round(64 * n / f / 1e6, 1),
            "inverse_in_place_ms": round(i, 4), "inverse_alg_GBps": round(64 * n / i / 1e6, 1)}


def spectral_512(torch, np, time_fn, warmup, steps):
    """Spectral operators on the 512^3 FP32 R2C plan (the Poisson right-hand
    side recipe as input): Laplacian (five passes with the fused x-pass),
    gradient (forward once, three fused multiplies and inverses) and
    divergence (three forwards and fused multiplies, one inverse).
    Algorithmic bytes, R = real field, H = half spectrum: Laplacian 2R + 8H,
    gradient 4R + 18H, divergence 4R + 20H."""
    from paper_1506_07933_amd import Plan, synth
    from paper_1506_07933_amd._lib import MIFFT_OP_LAPLACIAN
    n = 512
    p = Plan((n, n, n), "r2c", "fp32")
    f = synth.poisson_rhs_torch(n, 0, torch.float32, "cuda")
    v = [synth.poisson_rhs_torch(n, s, torch.float32, "cuda") for s in (1, 2, 3)]
    ws = torch.empty(p.spectral_ws_bytes, dtype=torch.uint8, device="cuda")
    u = torch.empty_like(f)
    g = [torch.empty_like(f) for _ in range(3)]
    lap = time_fn(lambda: p.spectral(MIFFT_OP_LAPLACIAN, f, out=u, ws=ws), warmup, steps)
    grad = time_fn(lambda: p.gradient(f, outs=g, ws=ws), warmup, steps)
    div = time_fn(lambda: p.divergence(v, out=u, ws=ws), warmup, steps)
    p.close()
    R = 4.0 * n ** 3
    H = 8.0 * n * n * (n // 2 + 1)
    return {"laplacian_ms": round(lap, 4), "laplacian_alg_GBps": round((2 * R + 8 * H) / lap / 1e6, 1),
            "gradient_ms": round(grad, 4), "gradient_alg_GBps": round((4 * R + 18 * H) / grad / 1e6, 1),
            "divergence_ms": round(div, 4), "divergence_alg_GBps": round((4 * R + 20 * H) / div / 1e6, 1)}


def cpu_baseline_configs(np, reps=3):
    """The oracle (unchanged) timed on the host's cores for the other
    workloads, median of `reps` runs on the same input, FP64, as context beside
    the GPU times: 32^3 C2C forward + inverse; 256^3 R2C forward; one pencil
    share 256 x 256 x 1024 (z-DFT, pack, loopback, unpack, y-DFT); the 64
    uneven transforms; one Poisson solve per served size (one run for 384^3
    and 512^3)."""
    import statistics
    import oracle
    from paper_1506_07933_amd import synth

    def med(fn, n=reps):
        ts = []
        for _ in range(n):
            t0 = time.perf_counter()
            fn()
            ts.append(time.perf_counter() - t0)
        print("oracle: %.1f ms" % (statistics.median(ts) * 1e3), file=sys.stderr, flush=True)
        return round(statistics.median(ts) * 1e3, 2)

    out = {"cores": oracle.max_threads(), "unit": "ms", "reps": reps}
    x = synth.uniform_complex((32, 32, 32), np.complex128, seed=0)
    out["c2c_32cube_fwd_inv"] = med(lambda: oracle.fft3d_c2c(oracle.fft3d_c2c(x, -1), +1))
    r = synth.normal_real((256, 256, 256), np.float64, seed=0)
    out["r2c_256cube_fwd"] = med(lambda: oracle.fft3d_r2c(r))
    a = synth.uniform_complex((256, 256, 1024), np.complex128, seed=0)
    out["pencil_share_256x256x1024"] = med(lambda: oracle.pencil_share_forward(a, 4))
    del a
    shapes, data = synth.batched_uneven(64, seed=0, dtype=np.complex128)
    out["batched_64_uneven"] = med(lambda: [oracle.fft3d_c2c(d, -1) for d in data])
    del data
    for n in (64, 128, 256, 384, 512):
        f, _ = synth.poisson_rhs(n, seed=0)
        out["poisson_%dcube" % n] = med(lambda: oracle.poisson_solve(f), reps if n < 384 else 1)
    return out


def pattern_mode(torch, time_fn, warmup, steps):
    """Copy rates of the strided passes' access pattern with no arithmetic
    (mifft_pattern_copy): the 512^3 y- and x-pass geometry -- 512 groups of
    512 columns, rows read 4 KiB apart and written 2 MiB apart (the
    transposing schedule) -- for several tile shapes, next to a plain
    contiguous device copy.  The ceiling the strided FFT passes are read
    against."""
    from paper_1506_07933_amd._lib import check, lib
    n = 512 ** 3
    a = torch.empty(n, dtype=torch.complex64, device="cuda")
    a.real.uniform_()
    b = torch.empty_like(a)
    out = {}
    for B, T in ((32, 32), (32, 16), (64, 16), (16, 64), (128, 8)):
        def run():
            check(lib.mifft_pattern_copy(0, a.data_ptr(), n, b.data_ptr(), n, 512, 512, 512, 512, 512 * 512,
                                         512 * 512, 512, B, T, 3, torch.cuda.current_stream().cuda_stream),
                  "mifft_pattern_copy")
        ms = time_fn(run, warmup, steps)
        out["tile_B%d_T%d_GBps" % (B, T)] = round(16 * n / ms / 1e6, 1)
    ms = time_fn(lambda: b.copy_(a), warmup, steps)
    out["contiguous_copy_GBps"] = round(16 * n / ms / 1e6, 1)
    return out


def workload_mode(args):
    """One secondary workload alone (for rocprofv3): the 64 uneven transforms
    in one persistent graph launch and as per-pass kernels, 512^3 R2C
    Poisson solves (FP32 and FP64), one task's 512^3 slab share, the 4-D
    512 x 256 x 128 x 64 C2C transform, the 512^3 spectral operators, one
    GPU's pencil share of a 1024^3 transform, the 256^3 R2C / C2R
    transforms, or the full served-Poisson replay."""
    import numpy as np
    import torch

    from paper_1506_07933_amd import BatchPlan, Plan, synth
    time_fn = _timer(torch)
    out = {"mode": args.mode}
    if args.mode == "batched":
        shapes, data = synth.batched_uneven(64, seed=0, dtype=np.complex64)
        xs = [torch.from_numpy(d).cuda() for d in data]
        outs = [torch.empty_like(v) for v in xs]
        bp = BatchPlan(shapes, "fp32")
        out["persistent_graph_ms"] = time_fn(lambda: bp.forward(xs, outs, graph=True), args.warmup, args.steps)
        assert not bp.aborted()
        bt = BatchPlan(shapes, "fp32", tune=True)
        out["persistent_tuned_graph_ms"] = time_fn(lambda: bt.forward(xs, outs, graph=True), args.warmup, args.steps)
        assert not bt.aborted()
        out["tuned_choices"] = [l for l in bt.describe().splitlines() if l.startswith("stage=")]
        bt.close()
        bk = BatchPlan(shapes, "fp32", mode="kernels")
        out["per_pass_kernels_ms"] = time_fn(lambda: bk.forward(xs, outs), args.warmup, args.steps)
        bg = BatchPlan(shapes, "fp32", mode="grouped")
        out["grouped_graph_ms"] = time_fn(lambda: bg.forward(xs, outs, graph=True), args.warmup, args.steps)
        bp.close()
        bk.close()
        bg.close()
    elif args.mode == "slab":
        out.update(slab_share(torch, np, time_fn, args.warmup, args.steps))
    elif args.mode == "nd":
        out.update(nd_4d(torch, time_fn, args.warmup, args.steps))
    elif args.mode == "spectral":
        out.update(spectral_512(torch, np, time_fn, args.warmup, args.steps))
    elif args.mode == "pattern":
        out.update(pattern_mode(torch, time_fn, args.warmup, args.steps))
    elif args.mode == "oracle":
        out.update(cpu_baseline_configs(np))
    elif args.mode == "pencil":
        # one GPU's share of a 1024^3 C2C transform on a 4 x 4 grid: the fused
        # z-FFT + pack and unpack + y-FFT kernels
        from paper_1506_07933_amd import PencilPlan
        pp = PencilPlan((1024, 1024, 1024), (4, 4), "fp32")
        a = torch.from_numpy(synth.uniform_complex(pp.local_shape, np.complex64, seed=0)).cuda()
        send = torch.empty(pp.send_shape, dtype=torch.complex64, device="cuda")
        ob = torch.empty(pp.out_shape, dtype=torch.complex64, device="cuda")
        out["pencil_share_fused_ms"] = time_fn(lambda: pp.forward_share(a, send, ob, fused=True), args.warmup,
                                               args.steps)
        pp.close()
    elif args.mode == "r2c":
        # 256^3 R2C forward and C2R inverse, FP32 and FP64
        for prec, rd, cd in (("fp32", np.float32, torch.complex64), ("fp64", np.float64, torch.complex128)):
            xr = torch.from_numpy(synth.normal_real((256, 256, 256), rd, seed=0)).cuda()
            p = Plan((256, 256, 256), "r2c", prec)
            Y = torch.empty((256, 256, 129), dtype=cd, device="cuda")
            xo = torch.empty_like(xr)
            out["r2c_256_%s_forward_ms" % prec] = time_fn(lambda: p.forward(xr, out=Y), args.warmup, args.steps)
            out["r2c_256_%s_inverse_ms" % prec] = time_fn(lambda: p.inverse(Y, out=xo), args.warmup, args.steps)
            p.close()
    elif args.mode == "serve":
        # the full served-Poisson replay: 2000 requests at 200 req/s (about 10 s)
        from paper_1506_07933_amd import serve
        s, _, ex = serve.serve(n_requests=2000, rate=200.0, seed=0, slots=4, budget_gb=32.0)
        ex.close()
        out.update({k: (round(v, 4) if isinstance(v, float) else v) for k, v in s.items()})
    else:
        for prec, dt in (("fp32", np.float32), ("fp64", np.float64)):
            f, _ = synth.poisson_rhs(512, seed=0, dtype=dt)
            fd = torch.from_numpy(f).cuda()
            p = Plan((512, 512, 512), "r2c", prec)
            u = torch.empty_like(fd)
            ws = torch.empty(p.poisson_ws_bytes, dtype=torch.uint8, device="cuda")
            out["poisson_512_%s_ms" % prec] = time_fn(lambda: p.poisson(fd, out=u, ws=ws), args.warmup, args.steps)
            p.close()
            del fd, u, ws
    print(json.dumps({k: (round(v, 4) if isinstance(v, float) else v) for k, v in out.items()}), flush=True)


def copy_ceiling(torch, x):
    """The best plain copy of the tensor x's bytes on this device: the
    library's reference copy (16-byte words, cached or streaming loads and
    stores, one pass or a grid-stride loop over CUs x 8 workgroups) and
    torch's copy_; returns (best GB/s, which, torch GB/s)."""
    from paper_1506_07933_amd._lib import lib
    y = torch.empty_like(x)
    nbytes = x.numel() * x.element_size()
    t = _timer(torch)
    torch_ms = t(lambda: y.copy_(x), 2, 10)
    best, kind = 2 * nbytes / (torch_ms * 1e-3) / 1e9, "torch copy_"
    cus = torch.cuda.get_device_properties(0).multi_processor_count
    names = {0: "cached", 1: "streaming loads", 2: "streaming stores", 3: "streaming loads and stores"}
    for flags in (0, 1, 2, 3, 4, 5, 6, 7):
        for grid in ((0,) if flags & 4 else (0, 8 * cus)):
            def run():
                rc = lib.mifft_copy_reference(x.data_ptr(), y.data_ptr(), nbytes, flags, grid, None)
                if rc:
                    raise RuntimeError(lib.mifft_last_error().decode())
            ms = t(run, 2, 10)
            gbs = 2 * nbytes / (ms * 1e-3) / 1e9
            if gbs > best:
                best, kind = gbs, "mifft_copy_reference, %s, %s" % (
                    names[flags & 3], "8 KiB blocks" if flags & 4 else
                    ("one pass" if grid == 0 else "grid of %d" % grid))
    torch_gbs = 2 * nbytes / (torch_ms * 1e-3) / 1e9
    del y
    return best, kind, torch_gbs


def oracle_one_thread(timeout_s: int = 240):
    """Seconds the oracle takes for the 512^3 forward transform of the same
    input on one thread (a child process with OMP_NUM_THREADS=1), or None."""
    import subprocess
    code = ("import time, numpy as np, oracle\n"
            "from paper_1506_07933_amd import synth\n"
            "x = synth.uniform_complex((%d, %d, %d), np.complex64, seed=0).astype(np.complex128)\n"
            "assert oracle.max_threads() == 1\n"
            "t0 = time.perf_counter(); oracle.fft3d_c2c(x, -1); print(time.perf_counter() - t0)\n" % (N0, N1, N2))
    env = dict(os.environ, OMP_NUM_THREADS="1")
    try:
        r = subprocess.run([sys.executable, "-c", code], cwd=ROOT, env=env, capture_output=True, text=True,
                           timeout=timeout_s)
        return round(float(r.stdout.strip().splitlines()[-1]), 3) if r.returncode == 0 else None
    except (subprocess.TimeoutExpired, ValueError, IndexError):
        return None


# Least device time every timed workload runs untimed first: the device drops
# out of its steady state while the host prepares the next workload's inputs
# (the pencil share measured 0.444 ms after 2 warm-up calls there, 0.388 ms
# after 100 in a process of its own).
MIN_WARM_S = 0.1


def _timer(torch):
    def time_fn(fn, warmup, steps):
        t0 = time.perf_counter()
        n = 0
        while n < warmup or time.perf_counter() - t0 < MIN_WARM_S:
            fn()
            n += 1
            if n % 8 == 0:
                torch.cuda.synchronize()
        torch.cuda.synchronize()
        a = torch.cuda.Event(enable_timing=True)
        b = torch.cuda.Event(enable_timing=True)
        a.record()
        for _ in range(steps):
            fn()
        b.record()
        torch.cuda.synchronize()
        return a.elapsed_time(b) / steps
    return time_fn


def secondary(torch, np, steps):
    """Short measurements of the other workloads (context for the headline)."""
    from paper_1506_07933_amd import BatchPlan, PencilPlan, Plan, serve, synth
    time_fn = _timer(torch)
    out = {}
    # plain single-transform FP64 path at the headline size
    x = torch.from_numpy(synth.uniform_complex((512, 512, 512), np.complex128, seed=0)).cuda()
    y = torch.empty_like(x)
    p = Plan((512, 512, 512), "c2c", "fp64")
    ms = time_fn(lambda: p.forward(x, out=y), 2, max(3, steps // 4))
    out["c2c_512cube_fp64_forward"] = {"ms": round(ms, 4), "alg_GBps": round(48 * 2 * 512 ** 3 / ms / 1e6, 1)}
    p.close()
    del x, y
    # 32^3 complex128 forward + inverse (latency-bound)
    x = torch.from_numpy(synth.uniform_complex((32, 32, 32), np.complex128, seed=0)).cuda()
    y = torch.empty_like(x)
    p = Plan((32, 32, 32), "c2c", "fp64")
    ms = time_fn(lambda: (p.forward(x, out=y), p.inverse(y, out=y)), 5, max(10, steps))
    out["c2c_32cube_fp64_forward_inverse"] = {"us": round(ms * 1e3, 2)}
    p.close()
    # 256^3 R2C / C2R, FP64 and FP32
    for prec, rd, cd in (("fp64", np.float64, torch.complex128), ("fp32", np.float32, torch.complex64)):
        xr = torch.from_numpy(synth.normal_real((256, 256, 256), rd, seed=0)).cuda()
        p = Plan((256, 256, 256), "r2c", prec)
        Y = torch.empty((256, 256, 129), dtype=cd, device="cuda")
        xo = torch.empty_like(xr)
        f = time_fn(lambda: p.forward(xr, out=Y), 2, steps)
        i = time_fn(lambda: p.inverse(Y, out=xo), 2, steps)
        esz = 8 if prec == "fp64" else 4
        alg = 256 ** 3 * esz + 5 * 256 * 256 * 129 * 2 * esz
        out["r2c_256cube_" + prec] = {"forward_ms": round(f, 4), "inverse_ms": round(i, 4),
                                      "forward_alg_GBps": round(alg / f / 1e6, 1)}
        p.close()
    # one GPU's pencil share of a 1024^3 transform on a 4x4 grid
    pp = PencilPlan((1024, 1024, 1024), (4, 4), "fp32")
    a = torch.from_numpy(synth.uniform_complex(pp.local_shape, np.complex64, seed=0)).cuda()
    send = torch.empty(pp.send_shape, dtype=torch.complex64, device="cuda")
    ob = torch.empty(pp.out_shape, dtype=torch.complex64, device="cuda")
    nl = a.numel()
    fused = time_fn(lambda: pp.forward_share(a, send, ob, fused=True), 2, steps)
    unfused = time_fn(lambda: pp.forward_share(a.clone(), send, ob, fused=False), 1, max(3, steps // 4))
    out["pencil_share_256x256x1024_fp32"] = {
        "fused_ms": round(fused, 4), "fused_alg_GBps": round(32 * nl / fused / 1e6, 1),
        "unfused_ms_incl_input_copy": round(unfused, 4)}
    pp.close()
    del a, send, ob
    out["slab_share_512cube_p4_fp32"] = slab_share(torch, np, time_fn, 2, steps)
    out["c2c_4d_512x256x128x64_fp32"] = nd_4d(torch, time_fn, 2, max(3, steps // 4))
    out["spectral_512cube_fp32"] = spectral_512(torch, np, time_fn, 2, max(3, steps // 2))
    # 64 uneven transforms: one persistent graph launch, per-pass kernels, and
    # one launch per pass and shape (in a graph)
    shapes, data = synth.batched_uneven(64, seed=0, dtype=np.complex64)
    xs = [torch.from_numpy(d).cuda() for d in data]
    outs = [torch.empty_like(v) for v in xs]
    nb = sum(v.numel() for v in xs)
    bp = BatchPlan(shapes, "fp32")
    g = time_fn(lambda: bp.forward(xs, outs, graph=True), 2, steps)
    assert not bp.aborted()
    bt = BatchPlan(shapes, "fp32", tune=True)
    gt = time_fn(lambda: bt.forward(xs, outs, graph=True), 2, steps)
    assert not bt.aborted()
    bk = BatchPlan(shapes, "fp32", mode="kernels")
    k = time_fn(lambda: bk.forward(xs, outs), 2, steps)
    bg = BatchPlan(shapes, "fp32", mode="grouped")
    gg = time_fn(lambda: bg.forward(xs, outs, graph=True), 2, steps)
    out["batched_64_uneven_fp32"] = {"persistent_graph_ms": round(g, 4), "persistent_tuned_graph_ms": round(gt, 4),
                                     "per_pass_kernels_ms": round(k, 4),
                                     "grouped_graph_ms": round(gg, 4), "elements": nb,
                                     "persistent_alg_GBps": round(48 * nb / g / 1e6, 1),
                                     "grouped_alg_GBps": round(48 * nb / gg / 1e6, 1)}
    bp.close()
    bt.close()
    bk.close()
    bg.close()
    del xs, outs
    # served Poisson solves: the configured open-loop replay (2000 requests at
    # 200 req/s, about 10 s), then 300 of them under a budget small enough
    # that admission has to queue requests
    for key, nreq, budget in (("served_poisson", 2000, 32.0), ("served_poisson_budget_5GB", 300, 5.0)):
        s, recs, ex = serve.serve(n_requests=nreq, rate=200.0, seed=0, slots=4, budget_gb=budget)
        ex.close()
        out[key] = {k2: (round(v, 4) if isinstance(v, float) else v) for k2, v in s.items()}
    return out


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    # Untimed warm-up: the MI355X reaches its steady memory throughput only after
    # tens of milliseconds of sustained load (the 512^3 strided passes take
    # 424 us in the first ~30 ms of a process, 400 us after 50 warm-up steps).
    ap.add_argument("--warmup", type=int, default=100)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-secondary", action="store_true")
    ap.add_argument("--mode", choices=["fft", "copy", "batched", "poisson", "slab", "nd", "spectral", "serve", "oracle",
                                       "pattern", "pencil", "r2c"], default="fft",
                    help="copy: plain 1 GiB device copy (counter scaling); batched / poisson / "
                         "slab / nd / spectral / pencil / r2c / serve: only that secondary workload (serve: the "
                         "full 2000-request replay); oracle: the CPU oracle's times for those "
                         "workloads; pattern: copy rates of the strided passes' access pattern")
    args = ap.parse_args()
    world = int(os.environ.get("WORLD_SIZE", "1"))
    if args.gpus != 1 or world != 1:
        print("bench.py measures one GPU: the local FFT phases run on a single MI355X and the "
              "library has no multi-GPU exchange; run it with --gpus 1", file=sys.stderr)
        sys.exit(2)
    if args.mode == "copy":
        return copy_mode(args)
    if args.mode in ("batched", "poisson", "slab", "nd", "spectral", "serve", "oracle", "pattern", "pencil", "r2c"):
        return workload_mode(args)

    import numpy as np
    import torch

    from paper_1506_07933_amd import Plan, synth
    from paper_1506_07933_amd.fft import profile_begin, profile_end

    n = N0 * N1 * N2
    x_host = synth.uniform_complex((N0, N1, N2), np.complex64, seed=0)
    x = torch.from_numpy(x_host).to("cuda:0")
    y = torch.empty_like(x)
    plan = Plan((N0, N1, N2), "c2c", "fp32")
    passes = [l for l in plan.describe().splitlines() if l.startswith("forward ")]
    axes = [l.split("axis=")[1][0] for l in passes]

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
    pass_ms, ncalls = profile_end(plan.handle, max_passes=64)
    ms = start.elapsed_time(stop) / args.steps
    # the same steps timed one by one (after the timed region), for the
    # median and the minimum per step
    ev = [torch.cuda.Event(enable_timing=True) for _ in range(args.steps + 1)]
    ev[0].record()
    for i in range(args.steps):
        plan.forward(x, out=y)
        ev[i + 1].record()
    torch.cuda.synchronize()
    per_step = sorted(ev[i].elapsed_time(ev[i + 1]) for i in range(args.steps))
    ms_median = per_step[len(per_step) // 2] if len(per_step) % 2 else \
        0.5 * (per_step[len(per_step) // 2 - 1] + per_step[len(per_step) // 2])

    # the copy ceiling: the best plain device copy of the same 1 GiB
    copy_best, copy_kind, torch_copy_GBps = copy_ceiling(torch, x)

    total_bytes = 3 * 16 * n  # 48 N: each pass reads and writes every complex64 once
    value = total_bytes / (ms * 1e-3) / 1e9
    kbytes = 16 * n  # one axis pass: read + write of N complex64
    per_axis = {}
    for a, t in zip(axes, pass_ms):
        per_axis[a] = per_axis.get(a, 0.0) + t
    names = {"z": "z_contig", "y": "y_strided", "x": "x_strided"}
    dom = max(per_axis, key=per_axis.get)
    launches = sum(1 for a in axes if a == dom)
    achieved = kbytes / (per_axis[dom] * 1e-3) / 1e9
    kname = {"z": "k_contig", "y": "k_strided(y, transposing)", "x": "k_strided(x)"}[dom]
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
        "device_copy_GBps": round(copy_best, 1),
        "device_copy_kind": copy_kind,
        "torch_copy_GBps": round(torch_copy_GBps, 1),
        "frac_of_device_copy": round(value / copy_best, 4),
        "wall_ms_per_step": round(wall * 1e3 / args.steps, 5),
        "ms_per_step_median": round(ms_median, 5),
        "ms_per_step_min": round(per_step[0], 5),
        "passes": [{"pass": names[a], "ms": round(per_axis[a], 5), "launches": axes.count(a),
                    "alg_GBps": round(kbytes / (per_axis[a] * 1e-3) / 1e9, 1),
                    "frac_of_hbm_peak": round(kbytes / (per_axis[a] * 1e-3) / 1e9 / PEAK_HBM_GBS, 4),
                    "frac_of_device_copy": round(kbytes / (per_axis[a] * 1e-3) / 1e9 / copy_best, 4)}
                   for a in "zyx" if a in per_axis],
        "plan": passes,
        "roofline": {"bound": "hbm", "kernel": kname + " " + names[dom],
                     "achieved": round(achieved, 1), "peak": PEAK_HBM_GBS, "unit": "GB/s",
                     "frac": round(achieved / PEAK_HBM_GBS, 4), "traffic": traffic,
                     "frac_of_device_copy": round(achieved / copy_best, 4),
                     "alg_bytes_per_axis_pass": kbytes, "launches_per_step": launches,
                     "steps_timed": ncalls,
                     # counter bytes over the same measured launch duration (DRAM rate)
                     "traffic_GBps": (round(traffic * launches / (per_axis[dom] * 1e-3) / 1e9, 1)
                                      if traffic else None)},
    }
    if not args.no_cpu_baseline:
        import oracle
        x64 = x_host.astype(np.complex128)
        runs = []
        for _ in range(3):
            t0 = time.perf_counter()
            ref = oracle.fft3d_c2c(x64, -1)
            runs.append(time.perf_counter() - t0)
        t_cpu = sorted(runs)[1]
        got = y.cpu().numpy().astype(np.complex128)
        rel = float(np.linalg.norm(got - ref) / np.linalg.norm(ref))
        del ref, got
        one = oracle_one_thread()
        out["cpu_baseline"] = {"value": round(total_bytes / t_cpu / 1e9, 3), "unit": "GB/s",
                               "cores": oracle.max_threads(), "kind": "oracle",
                               "sample": "the full 512^3 forward transform of the same input, FP64, "
                                         "median of 3 runs (%s s)" % ", ".join("%.2f" % r for r in runs),
                               "median_s": round(t_cpu, 3),
                               "one_thread_s": one,
                               "one_thread_GBps": round(total_bytes / one / 1e9, 3) if one else None}
        out["rel_l2_vs_oracle"] = rel
    plan.close()
    del x, y
    if not args.no_secondary:
        torch.cuda.empty_cache()
        out["secondary"] = secondary(torch, np, args.steps)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
