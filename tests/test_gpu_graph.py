"""Single-transform execute calls captured into a HIP graph (torch.cuda.CUDAGraph
over the library's C calls): the calls only enqueue kernels, allocate
nothing and never synchronise, so they can be captured.  Every replay, with
eager work on the same buffers in between, must equal the eager result bit
for bit."""
import numpy as np
import pytest

import oracle
from paper_1506_07933_amd import synth
from conftest import TOL, rel_l2

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu


def _replays_equal(run, outputs, reps=4):
    """Eager reference, capture, then `reps` replays each compared bit for bit;
    between replays the outputs are overwritten eagerly."""
    torch.cuda.synchronize()
    run()
    torch.cuda.synchronize()
    ref = [o.clone() for o in outputs]
    g = torch.cuda.CUDAGraph()
    s = torch.cuda.Stream()
    s.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(s):
        run()  # warm-up on the capture stream
    torch.cuda.current_stream().wait_stream(s)
    torch.cuda.synchronize()
    with torch.cuda.graph(g):
        run()
    for r in range(reps):
        for o in outputs:
            o.fill_(float(r + 7))  # eager work between replays
        g.replay()
        torch.cuda.synchronize()
        for o, e in zip(outputs, ref):
            assert torch.equal(o, e), "replay %d differs" % r
    return ref


def test_c2c_forward_inverse_graph():
    from paper_1506_07933_amd import Plan
    shape = (64, 96, 128)
    x = torch.from_numpy(synth.uniform_complex(shape, np.complex64, seed=5)).cuda()
    y = torch.empty_like(x)
    z = torch.empty_like(x)
    p = Plan(shape, "c2c", "fp32")

    def run():
        p.forward(x, out=y)
        p.inverse(y, out=z)

    ref = _replays_equal(run, [y, z])
    x64 = x.cpu().numpy().astype(np.complex128)
    assert rel_l2(ref[0].cpu().numpy(), oracle.fft3d_c2c(x64, -1)) <= TOL["fp32"]
    assert rel_l2(ref[1].cpu().numpy(), np.prod(shape) * x64) <= TOL["fp32"]
    p.close()


@pytest.mark.parametrize("prec", ["fp32", "fp64"])
def test_poisson_graph_transposed(prec):
    """A 128 x 256 x 256 Poisson solve (transposed intermediate, padded rows,
    fused x-pass) with a caller-owned workspace, captured and replayed."""
    from paper_1506_07933_amd import Plan
    shape = (128, 256, 256)
    rd = np.float32 if prec == "fp32" else np.float64
    f64 = synth.normal_real(shape, np.float64, seed=6)
    f64 -= f64.mean()
    f = torch.from_numpy(f64.astype(rd)).cuda()
    u = torch.empty_like(f)
    p = Plan(shape, "r2c", prec)
    ws = torch.empty(p.poisson_ws_bytes, dtype=torch.uint8, device="cuda")

    def run():
        p.poisson(f, out=u, ws=ws)

    (ref,) = _replays_equal(run, [u])
    assert rel_l2(ref.cpu().numpy(), oracle.poisson_solve(f.cpu().numpy().astype(np.float64))) <= TOL[prec]
    p.close()


def test_poisson_graph_with_the_side_stream(monkeypatch):
    """A 512^3 FP32 solve runs the Nyquist plane's passes on a side stream
    (fork after the z-pass, join before the C2R).  Captured on a stream that
    already has its side stream (an eager call on it first), the graph holds
    both branches: every replay equals the eager result bit for bit, and so
    does the solve with every pass in line (same kernels on the same data)."""
    from paper_1506_07933_amd import Plan
    shape = (512, 512, 512)
    f64 = synth.normal_real(shape, np.float64, seed=9)
    f = torch.from_numpy((f64 - f64.mean()).astype(np.float32)).cuda()
    del f64
    u = torch.empty_like(f)
    p = Plan(shape, "r2c", "fp32")
    assert "fork=1" in p.describe() and "join=1" in p.describe()
    ws = torch.empty(p.poisson_ws_bytes, dtype=torch.uint8, device="cuda")
    s = torch.cuda.Stream()
    s.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(s):
        p.poisson(f, out=u, ws=ws)  # creates the side stream of s
    s.synchronize()
    ref = u.clone()
    monkeypatch.setenv("MIFFT_SIDE_STREAM", "0")
    u.fill_(3.0)
    p.poisson(f, out=u, ws=ws)
    torch.cuda.synchronize()
    assert torch.equal(u, ref), "in-line solve differs"
    monkeypatch.delenv("MIFFT_SIDE_STREAM")
    g = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g, stream=s):
        p.poisson(f, out=u, ws=ws)
    for r in range(3):
        u.fill_(float(r + 7))  # eager work between replays
        g.replay()
        torch.cuda.synchronize()
        assert torch.equal(u, ref), "replay %d differs" % r
    # captured on a stream that has made no call before (it takes its side
    # stream from the plan's pool inside the capture)
    g2 = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g2):
        p.poisson(f, out=u, ws=ws)
    for r in range(2):
        u.fill_(float(r + 11))
        g2.replay()
        torch.cuda.synchronize()
        assert torch.equal(u, ref), "replay %d of the second graph differs" % r
    del g, g2
    p.close()


def test_poisson_side_streams_per_caller_stream():
    """A 512^3 FP32 plan holds four side streams; calls on five distinct
    caller streams (the fifth runs the plane's passes in line) and on the
    default stream all give the same result bit for bit."""
    from paper_1506_07933_amd import Plan
    shape = (512, 512, 512)
    f = torch.empty(shape, dtype=torch.float32, device="cuda")
    synth.poisson_rhs_device(f, seed=3)
    u = torch.empty_like(f)
    p = Plan(shape, "r2c", "fp32")
    ws = torch.empty(p.poisson_ws_bytes, dtype=torch.uint8, device="cuda")
    p.poisson(f, out=u, ws=ws)
    torch.cuda.synchronize()
    ref = u.clone()
    streams = [torch.cuda.Stream() for _ in range(5)]
    for i, st in enumerate(streams):
        st.wait_stream(torch.cuda.current_stream())
        with torch.cuda.stream(st):
            u.fill_(float(i + 1))
            p.poisson(f, out=u, ws=ws)
        st.synchronize()
        assert torch.equal(u, ref), "stream %d differs" % i
    p.close()


def test_spectral_gradient_divergence_graph():
    """Gradient and divergence (several launches over a caller workspace)
    captured together and replayed."""
    from paper_1506_07933_amd import Plan
    shape = (64, 256, 256)
    f = torch.from_numpy(synth.normal_real(shape, np.float32, seed=7)).cuda()
    v = [torch.from_numpy(synth.normal_real(shape, np.float32, seed=8 + j)).cuda() for j in range(3)]
    p = Plan(shape, "r2c", "fp32")
    ws = torch.empty(p.spectral_ws_bytes, dtype=torch.uint8, device="cuda")
    g = [torch.empty_like(f) for _ in range(3)]
    d = torch.empty_like(f)

    def run():
        p.gradient(f, outs=g, ws=ws)
        p.divergence(v, out=d, ws=ws)

    ref = _replays_equal(run, g + [d])
    want = oracle.gradient(f.cpu().numpy().astype(np.float64))
    for j in range(3):
        assert rel_l2(ref[j].cpu().numpy(), want[j]) <= TOL["fp32"]
    p.close()


def test_slab_and_nd_graph():
    """One task's slab stages (p = 2, the send buffer as the receive buffer) and a rank-4 plan's
    forward + inverse captured and replayed."""
    from paper_1506_07933_amd import Plan, SlabPlan
    sp = SlabPlan((32, 32, 32), 2, "c2c", "fp32")
    a = torch.from_numpy(synth.uniform_complex(sp.slab_shape, np.complex64, seed=9)).cuda()
    send = torch.empty(sp.send_shape, dtype=torch.complex64, device="cuda")
    mid = torch.empty(sp.mid_shape, dtype=torch.complex64, device="cuda")
    share = torch.empty(sp.share_shape, dtype=torch.complex64, device="cuda")
    nd = Plan((8, 12, 16, 20), "c2c", "fp64")
    x = torch.from_numpy(synth.uniform_complex((8, 12, 16, 20), np.complex128, seed=10)).cuda()
    y = torch.empty_like(x)
    z = torch.empty_like(x)

    def run():
        sp.forward_local(a, send, mid)
        sp.forward_x(send, share)  # the send buffer stands in for the received slab
        nd.forward(x, out=y)
        nd.inverse(y, out=z)

    ref = _replays_equal(run, [send, share, y, z])
    want = oracle.fftnd_c2c(x.cpu().numpy(), -1)
    assert rel_l2(ref[2].cpu().numpy(), want) <= TOL["fp64"]
    sp.close()
    nd.close()
