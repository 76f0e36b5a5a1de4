"""GPU parity of the batched uneven-size executor (one persistent launch for
many 3-D C2C transforms), through the C ABI binding, against the FP64 oracle
and against the single-transform plans.  Per-transform rel-L2 bars as for
single plans (5e-6 FP32, 1e-13 FP64)."""
import numpy as np
import pytest

import oracle
from paper_1506_07933_amd import synth
from conftest import TOL, rel_l2

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu
DEV = "cuda:0"


def run_batch(shapes, data, prec, mode="persistent", graph=False, reps=1):
    from paper_1506_07933_amd import BatchPlan
    bp = BatchPlan(shapes, prec, mode=mode)
    print("  ", bp.describe().strip(), flush=True)
    xs = [torch.from_numpy(d).to(DEV) for d in data]
    outs = [torch.empty_like(x) for x in xs]
    results = []
    for _ in range(reps):
        for o in outs:
            o.zero_()
        print("   launch (graph=%s)" % graph, flush=True)
        bp.forward(xs, outs, graph=graph)
        torch.cuda.synchronize()
        print("   done", flush=True)
        assert not bp.aborted()
        results.append([o.cpu().numpy() for o in outs])
    bp.close()
    return results


def test_batched_uneven_64_persistent():
    """64 transforms drawn by seed from {48^3, 64^3, 96^3, 128^3, 100x120x144,
    125^3}, complex64 N(0,1): one persistent launch; each transform against
    the oracle and against its single-plan GPU result."""
    from paper_1506_07933_amd import Plan
    shapes, data = synth.batched_uneven(64, seed=0, dtype=np.complex64)
    (res,) = run_batch(shapes, data, "fp32")
    worst = 0.0
    plans = {}
    for i, (s, d, r) in enumerate(zip(shapes, data, res)):
        e = rel_l2(r, oracle.fft3d_c2c(d.astype(np.complex128), -1))
        worst = max(worst, e)
        assert e <= 5e-6, (i, s, e)
        if s not in plans:
            plans[s] = Plan(s, "c2c", "fp32")
        single = plans[s].forward(torch.from_numpy(d).to(DEV)).cpu().numpy()
        assert rel_l2(r, single) <= 5e-6, (i, s)
    print("  64 uneven transforms, worst rel_l2 vs oracle %.3e" % worst, flush=True)


def test_batch_graph_replays_match_eager():
    """The graph is replayed several times with eager work in between; every
    replay must equal the eager launch bit for bit."""
    shapes, data = synth.batched_uneven(12, seed=3, dtype=np.complex64)
    (eager,) = run_batch(shapes, data, "fp32")
    replays = run_batch(shapes, data, "fp32", graph=True, reps=4)
    for rep in replays:
        for a, b in zip(rep, eager):
            np.testing.assert_array_equal(a, b)


def test_batch_kernels_mode_and_fp64():
    shapes, data = synth.batched_uneven(10, seed=5, dtype=np.complex128)
    (res,) = run_batch(shapes, data, "fp64")
    (res_k,) = run_batch(shapes, data, "fp64", mode="kernels")
    for s, d, r, rk in zip(shapes, data, res, res_k):
        ref = oracle.fft3d_c2c(d, -1)
        assert rel_l2(r, ref) <= 1e-13, s
        assert rel_l2(rk, ref) <= 1e-13, s


@pytest.mark.parametrize("prec", ["fp32", "fp64"])
def test_batch_ragged_small_shapes(prec):
    """Lengths whose threads per line do not divide 64, 1-extents, in-place."""
    shapes = [(2, 3, 5), (1, 1, 256), (256, 1, 1), (1, 9, 1), (3, 125, 6), (12, 20, 15),
              (81, 2, 4), (5, 5, 5), (144, 1, 120), (2, 2, 2)]
    cd = np.complex64 if prec == "fp32" else np.complex128
    data = [synth.uniform_complex(s, cd, seed=i) for i, s in enumerate(shapes)]
    (res,) = run_batch(shapes, data, prec)
    for s, d, r in zip(shapes, data, res):
        assert rel_l2(r, oracle.fft3d_c2c(d.astype(np.complex128), -1)) <= TOL[prec], s
    # in place: in[t] == out[t]
    from paper_1506_07933_amd import BatchPlan
    bp = BatchPlan(shapes, prec)
    xs = [torch.from_numpy(d).to(DEV) for d in data]
    bp.forward(xs, xs)
    torch.cuda.synchronize()
    assert not bp.aborted()
    for x, r in zip(xs, res):
        np.testing.assert_array_equal(x.cpu().numpy(), r)
    bp.close()


def test_batch_grouped_mode():
    """MIFFT_BATCH_GROUPED: each pass of all transforms of one shape as one
    launch.  Same kernels and launch shapes as the per-pass mode, so the
    results are bit-identical to it; checked against the oracle too.  The
    shapes include 20 copies of one shape (two launches per pass), a 256^3
    transform whose plan uses a workspace (run per transform), 1x1x1 and
    ragged shapes."""
    rng = np.random.default_rng(71)
    shapes = [(32, 48, 40)] * 20 + [(256, 256, 256), (1, 1, 1), (5, 27, 6), (48, 64, 96)] * 2
    data = [(rng.standard_normal(s) + 1j * rng.standard_normal(s)).astype(np.complex64) for s in shapes]
    (res_g,) = run_batch(shapes, data, "fp32", mode="grouped")
    (res_k,) = run_batch(shapes, data, "fp32", mode="kernels")
    for t in range(len(shapes)):
        np.testing.assert_array_equal(res_g[t], res_k[t])
    for t in (0, 19, 20, 21, 22, 23):
        ref = oracle.fft3d_c2c(data[t].astype(np.complex128), -1)
        assert rel_l2(res_g[t], ref) <= TOL["fp32"], t
    # graph replay of the grouped launches
    (res_gg,) = run_batch(shapes, data, "fp32", mode="grouped", graph=True)
    for t in range(len(shapes)):
        np.testing.assert_array_equal(res_gg[t], res_g[t])


def test_batch_tuned_persistent_launch(tmp_path):
    """MIFFT_TUNE in the one persistent launch: per (stage, length) the tuner
    picks a code path (radix order, radix groups per thread) and an item
    size by timing the whole batch; the results keep parity with the oracle
    and with the untuned launch, the choices land in the wisdom file, and a
    second tuned batch of the same shapes reuses them."""
    import json
    import os
    from paper_1506_07933_amd import BatchPlan
    wisdom = tmp_path / "wisdom.json"
    os.environ["MIFFT_WISDOM"] = str(wisdom)
    try:
        shapes, data = synth.batched_uneven(16, seed=7, dtype=np.complex64)
        bp = BatchPlan(shapes, "fp32", tune=True)
        desc = bp.describe()
        print(desc, flush=True)
        assert "chosen" in desc
        xs = [torch.from_numpy(d).to(DEV) for d in data]
        outs = [torch.empty_like(x) for x in xs]
        bp.forward(xs, outs, graph=True)
        torch.cuda.synchronize()
        assert not bp.aborted()
        (plain,) = run_batch(shapes, data, "fp32")
        worst = 0.0
        for s, d, o, r in zip(shapes, data, outs, plain):
            got = o.cpu().numpy()
            e = rel_l2(got, oracle.fft3d_c2c(d.astype(np.complex128), -1))
            worst = max(worst, e)
            assert e <= 5e-6, s
            assert rel_l2(got, r) <= 5e-6, s
        print("  tuned batch worst rel_l2 vs oracle %.3e" % worst, flush=True)
        bp.close()
        entries = json.loads(wisdom.read_text())
        keys = [k for k in entries if "|batch_" in k]
        lengths = {n for s in shapes for n in s if n > 1}
        assert {k.split("|")[2] for k in keys} == {"batch_z", "batch_y", "batch_x"}
        assert {int(k.split("L=")[1]) for k in keys} == lengths
        for k in keys:
            pol, emul, kib, lpw, us = entries[k]
            assert pol in (0, 2) and emul in (1, 2) and kib in (32, 64, 128, 256) and lpw == 0 and us > 0
        again = BatchPlan(shapes, "fp32", tune=True)
        assert again.describe() == desc        # the stored choices, applied without timing
        again.close()
    finally:
        del os.environ["MIFFT_WISDOM"]
