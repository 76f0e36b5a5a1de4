"""GPU parity of the spectral operators (Laplacian, Helmholtz solve, partial
derivatives, gradient, divergence) on 3-D R2C plans, through the C ABI,
against the oracle's operators on the same inputs (rel-L2 <= 1e-13 FP64,
<= 5e-6 FP32).  Covered: the fused x-pass in the transposed and the standard
layout, the standalone multiply (n0 = 1, and MIFFT_POISSON_UNFUSED=1), odd
extents without a Nyquist mode, caller and plan workspaces, and argument
errors."""
import numpy as np
import pytest

import oracle
from paper_1506_07933_amd import synth
from conftest import TOL, rel_l2

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

DEV = "cuda:0"
RDT = {"fp32": np.float32, "fp64": np.float64}
OPS = [oracle.OP_POISSON, oracle.OP_LAPLACIAN, oracle.OP_HELMHOLTZ, oracle.OP_DX, oracle.OP_DY, oracle.OP_DZ]
# (shape, layout): 64 x 256 x 256 uses the transposed intermediate (x-stride
# 256 x 129 x 8 bytes >= 256 KiB), the others the standard layout; n0 = 1 runs
# the standalone multiply
SHAPES = [(64, 256, 256), (32, 24, 40), (27, 25, 30), (1, 32, 64), (16, 1, 24)]  # n1 = 1: no y-pass


def gpu(a):
    return torch.from_numpy(np.ascontiguousarray(a)).to(DEV)


def host(t):
    torch.cuda.synchronize()
    return t.cpu().numpy()


def report(name, err, tol):
    print("  %-56s rel_l2=%.3e (bar %.0e)" % (name, err, tol), flush=True)
    assert err <= tol, "%s: rel-L2 %.3e above %.0e" % (name, err, tol)


def _field(shape, prec, seed):
    f = synth.normal_real(shape, np.float64, seed=seed)
    return f.astype(RDT[prec])


@pytest.mark.parametrize("shape", SHAPES)
@pytest.mark.parametrize("prec", ["fp32", "fp64"])
def test_spectral_apply_every_operator(shape, prec):
    from paper_1506_07933_amd import Plan
    p = Plan(shape, "r2c", prec)
    f = _field(shape, prec, 61)
    fd = gpu(f)
    ws = torch.empty(p.poisson_ws_bytes, dtype=torch.uint8, device=DEV)
    f64 = f.astype(np.float64)
    for op in OPS:
        for alpha in ((0.0, 2.5) if op == oracle.OP_HELMHOLTZ else (0.0,)):
            u = p.spectral(op, fd, alpha=alpha, ws=ws)
            report("%s %s op %d alpha %.1f" % (shape, prec, op, alpha),
                   rel_l2(host(u), oracle.spectral_apply(f64, op, alpha)), TOL[prec])
    np.testing.assert_array_equal(host(fd), f)  # f preserved
    # the Poisson entry point is the POISSON operator, bit for bit
    assert torch.equal(p.poisson(fd, ws=ws), p.spectral(oracle.OP_POISSON, fd, ws=ws))
    p.close()


@pytest.mark.parametrize("shape", SHAPES)
@pytest.mark.parametrize("prec", ["fp32", "fp64"])
def test_gradient_and_divergence(shape, prec):
    from paper_1506_07933_amd import Plan
    p = Plan(shape, "r2c", prec)
    f = _field(shape, prec, 62)
    fd = gpu(f)
    ws = torch.empty(p.spectral_ws_bytes, dtype=torch.uint8, device=DEV)
    g = p.gradient(fd, ws=ws)
    ref = oracle.gradient(f.astype(np.float64))
    for j in range(3):
        report("%s %s gradient %d" % (shape, prec, j), rel_l2(host(g[j]), ref[j]), TOL[prec])
        # each component equals the single-derivative operator bit for bit
        assert torch.equal(g[j], p.spectral(oracle.OP_DX + j, fd))
    v = [gpu(_field(shape, prec, 63 + j)) for j in range(3)]
    d = p.divergence(v, ws=ws)
    refd = oracle.divergence(*[host(c).astype(np.float64) for c in v])
    report("%s %s divergence" % (shape, prec), rel_l2(host(d), refd), TOL[prec])
    d2 = p.divergence(v)  # the plan's own workspace
    assert torch.equal(d, d2)
    np.testing.assert_array_equal(host(fd), f)
    p.close()


@pytest.mark.parametrize("prec", ["fp32", "fp64"])
def test_unfused_multiply_path(monkeypatch, prec):
    """MIFFT_POISSON_UNFUSED=1 at plan time: forward transform, standalone
    multiply, inverse transform; same results within the bar."""
    from paper_1506_07933_amd import Plan
    monkeypatch.setenv("MIFFT_POISSON_UNFUSED", "1")
    shape = (64, 256, 256)
    p = Plan(shape, "r2c", prec)
    monkeypatch.delenv("MIFFT_POISSON_UNFUSED")
    f = _field(shape, prec, 64)
    fd = gpu(f)
    f64 = f.astype(np.float64)
    for op in (oracle.OP_LAPLACIAN, oracle.OP_HELMHOLTZ, oracle.OP_DZ):
        report("unfused %s op %d" % (prec, op), rel_l2(host(p.spectral(op, fd, alpha=1.0)),
                                                      oracle.spectral_apply(f64, op, 1.0)), TOL[prec])
    g = p.gradient(fd)
    ref = oracle.gradient(f64)
    for j in range(3):
        report("unfused %s gradient %d" % (prec, j), rel_l2(host(g[j]), ref[j]), TOL[prec])
    v = [gpu(_field(shape, prec, 65 + j)) for j in range(3)]
    report("unfused %s divergence" % prec,
           rel_l2(host(p.divergence(v)), oracle.divergence(*[host(c).astype(np.float64) for c in v])), TOL[prec])
    p.close()


def test_closed_form_modes_128():
    """Smooth mode sums at 128^3 FP64: gradient and Laplacian against the
    analytic derivatives."""
    from paper_1506_07933_amd import Plan
    n = 128
    ks, amp, phase, _ = synth.poisson_modes(n, seed=66)
    f = synth.mode_sum(n, ks, amp, phase)
    p = Plan((n, n, n), "r2c", "fp64")
    fd = gpu(f)
    g = p.gradient(fd)
    for j in range(3):
        report("128^3 gradient %d closed form" % j,
               rel_l2(host(g[j]), synth.mode_sum(n, ks, amp * ks[:, j], phase + np.pi / 2)), 1e-12)
    kk = np.sum(ks * ks, axis=1)
    report("128^3 Laplacian closed form",
           rel_l2(host(p.spectral(oracle.OP_LAPLACIAN, fd)), synth.mode_sum(n, ks, -amp * kk, phase)), 1e-12)
    p.close()


def test_spectral_errors():
    from paper_1506_07933_amd import Plan
    from paper_1506_07933_amd.fft import MifftError
    p = Plan((16, 16, 16), "r2c", "fp32")
    f = torch.zeros((16, 16, 16), dtype=torch.float32, device=DEV)
    u = torch.zeros_like(f)
    with pytest.raises(MifftError):
        p.spectral(6, f, out=u)          # unknown operator
    with pytest.raises(MifftError):
        p.spectral(1, f, out=f)          # aliased
    with pytest.raises(MifftError):
        p.gradient(f, outs=[u, u, torch.zeros_like(f)])
    with pytest.raises(MifftError):
        p.divergence([f, u, u], out=u)
    with pytest.raises(ValueError):
        p.gradient(f, ws=torch.empty(16, dtype=torch.uint8, device=DEV))
    c = Plan((16, 16, 16), "c2c", "fp32")
    with pytest.raises(MifftError):      # C2C plans have no spectral operators
        c.spectral(1, f, out=u)
    p.close()
    c.close()
