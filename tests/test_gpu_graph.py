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
