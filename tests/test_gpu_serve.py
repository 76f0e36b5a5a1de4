"""Served spectral Poisson solves on the GPU: an open-loop replay through the
continuous-batching scheduler.  Every request's result in the mix is compared
with the same request run alone (bit for bit: the same kernels run on the
same data) and, for every (size, precision) of the served mix, against the
FP64 oracle on the request's own right-hand side (per-request rel-L2 bars)."""
import numpy as np
import pytest

import oracle
from conftest import TOL, rel_l2

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

SIZES = (64, 128, 256, 384, 512)


def burst_schedule(seed=3, per_kind=2, gap=1e-3):
    """Every (size, precision) of the served mix `per_kind` times, in a
    seeded order, arriving 1 ms apart: faster than the solves complete, so
    requests overlap on the device and the budget makes some of them wait."""
    kinds = [(n, p) for n in SIZES for p in ("fp32", "fp64")] * per_kind
    order = np.random.default_rng(seed).permutation(len(kinds))
    return [(i * gap, kinds[k][0], kinds[k][1]) for i, k in enumerate(order)]


def test_served_poisson_mix_equals_alone_and_oracle():
    from paper_1506_07933_amd import serve
    budget_gb = 10.0
    sched = burst_schedule()
    summary, recs, ex = serve.serve(schedule=sched, seed=1, slots=3, budget_gb=budget_gb, keep_outputs=True)
    print("  ", {k: v for k, v in summary.items() if k != "timeline_t_queue_inflight_bytes"}, flush=True)
    assert summary["ok"] == len(sched) and summary["failed"] == 0 and summary["rejected"] == 0
    assert summary["peak_bytes_in_flight"] <= budget_gb * 2 ** 30
    assert summary["p99_ms"] >= summary["p50_ms"] > 0
    overlapped = sum(1 for r in recs.values() for q in recs.values()
                     if q.rid < r.rid and q.t_admit < r.t_done and r.t_admit < q.t_done)
    print("  overlapping request pairs:", overlapped, " max queue depth:", summary["max_queue_depth"],
          flush=True)
    assert overlapped > 0, "no two requests shared the device"
    assert summary["max_queue_depth"] > 0, "the budget / slots never made a request wait"
    checked = set()
    for rid, rec in sorted(recs.items()):
        req = serve.Request(rid, rec.t_arrival, rec.n, rec.prec)
        f_alone, u_alone = ex.run_alone(req)
        f_mix, u_mix = ex.inputs[rid], ex.outputs[rid]
        # the right-hand side is drawn from the request's seed: the same bits alone and in the mix
        assert torch.equal(f_mix, f_alone), "request %d: right-hand side differs" % rid
        assert torch.equal(u_mix, u_alone), "request %d: result in the mix differs from alone" % rid
        if (rec.n, rec.prec) not in checked:
            f = f_mix.cpu().numpy().astype(np.float64)
            e = rel_l2(u_mix.cpu().numpy(), oracle.poisson_solve(f))
            print("  request %d n=%d %s rel_l2 vs oracle %.3e (bar %.0e)" % (rid, rec.n, rec.prec, e,
                                                                          TOL[rec.prec]), flush=True)
            assert e <= TOL[rec.prec]
            checked.add((rec.n, rec.prec))
        del ex.inputs[rid], ex.outputs[rid]
    assert len(checked) == 2 * len(SIZES)
    ex.close()


def test_device_rhs_matches_the_host_recipe():
    """The served right-hand side drawn on the device has the mode part of
    the host recipe (noise off) to rounding, for both precisions."""
    from paper_1506_07933_amd import synth
    for n, dt, tol in ((64, torch.float64, 1e-12), (96, torch.float32, 1e-6)):
        f = torch.empty((n, n, n), dtype=dt, device="cuda")
        synth.poisson_rhs_device(f, seed=5, noise=0.0)
        ks, amp, ph, _ = synth.poisson_modes(n, 5)
        ref = synth.mode_sum(n, ks, amp, ph)
        e = rel_l2(f.cpu().numpy(), ref)
        print("  device rhs n=%d %s rel_l2 %.2e" % (n, dt, e), flush=True)
        assert e <= tol
        g = torch.empty_like(f)
        synth.poisson_rhs_device(g, seed=5)          # with noise: std about 0.01 around the modes
        d = (g - f).double()
        assert abs(float(d.std()) - 0.01) < 1e-3 and abs(float(d.mean())) < 1e-3
