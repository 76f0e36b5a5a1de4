"""GPU parity of transforms of rank other than 3 (Algorithm 2 with one task
per axis): the HIP path through mifft_plan_create_nd against the oracle's
N-D transforms (rel-L2 <= 1e-13 FP64, <= 5e-6 FP32), and the paper's 4-D
case 512 x 256 x 128 x 64 at full size against the sampled N-D definition
plus the round trip and Parseval over every element."""
import numpy as np
import pytest

import oracle
from oracle.brute import dftnd_at
from paper_1506_07933_amd import synth
from conftest import TOL, rel_l2

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

DEV = "cuda:0"
CDT = {"fp32": np.complex64, "fp64": np.complex128}
RDT = {"fp32": np.float32, "fp64": np.float64}


def gpu(a):
    return torch.from_numpy(np.ascontiguousarray(a)).to(DEV)


def host(t):
    torch.cuda.synchronize()
    return t.cpu().numpy()


def report(name, err, tol):
    print("  %-52s rel_l2=%.3e (bar %.0e)" % (name, err, tol), flush=True)
    assert err <= tol, "%s: rel-L2 %.3e above %.0e" % (name, err, tol)


C2C = [((8, 12, 10, 16), "fp32"), ((6, 5, 4, 3, 2), "fp64"), ((4, 1, 9, 8), "fp32"),
       ((2, 2, 2, 2, 2, 2, 2, 2), "fp64"), ((16, 32, 64, 128), "fp64"), ((1, 1, 1, 1), "fp32"),
       ((3, 27, 25, 1, 6), "fp32"), ((96,), "fp64"), ((48, 60), "fp32")]


@pytest.mark.parametrize("shape,prec", C2C)
def test_nd_c2c(shape, prec):
    from paper_1506_07933_amd import Plan
    p = Plan(shape, "c2c", prec)
    x = synth.uniform_complex(shape, CDT[prec], seed=51)
    xd = gpu(x)
    y = p.forward(xd)
    x64 = x.astype(np.complex128)
    report("nd %s %s forward" % (shape, prec), rel_l2(host(y), oracle.fftnd_c2c(x64, -1)), TOL[prec])
    z = p.inverse(y)
    report("nd %s %s inverse" % (shape, prec),
           rel_l2(host(z), oracle.fftnd_c2c(host(y).astype(np.complex128), +1)), TOL[prec])
    report("nd %s %s round trip" % (shape, prec), rel_l2(host(z), x.size * x64), TOL[prec])
    p.inverse(y, out=y)  # in place
    assert torch.equal(y, z)
    p.close()


# (8, 64, 32, 64) and (6, 40, 24, 48, 10): axis 0's stride is >= 256 KiB, so they run the
# transposed intermediate (and the R2C inverse's two workspace spectra)
R2C = [((8, 12, 10, 16), "fp32"), ((5, 4, 3, 6), "fp64"), ((3, 2, 2, 2, 2), "fp32"),
       ((2, 3, 4, 5, 6, 8), "fp64"), ((32, 16, 8, 64), "fp32"), ((40,), "fp64"), ((12, 30), "fp32"),
       ((8, 64, 32, 64), "fp32"), ((8, 64, 32, 64), "fp64"), ((6, 40, 24, 48, 10), "fp64")]


@pytest.mark.parametrize("shape,prec", R2C)
def test_nd_r2c_c2r(shape, prec):
    from paper_1506_07933_amd import Plan
    p = Plan(shape, "r2c", prec)
    x = synth.normal_real(shape, RDT[prec], seed=52)
    Y = p.forward(gpu(x))
    report("nd r2c %s %s forward" % (shape, prec), rel_l2(host(Y), oracle.fftnd_r2c(x.astype(np.float64))),
           TOL[prec])
    back = p.inverse(Y)
    report("nd r2c %s %s round trip" % (shape, prec), rel_l2(host(back), x.size * x.astype(np.float64)),
           TOL[prec])
    # non-Hermitian spectrum; the C2R keeps its input
    h = synth.uniform_complex(p.spec_shape, CDT[prec], seed=53)
    hd = gpu(h)
    out = p.inverse(hd)
    report("nd c2r %s %s non-Hermitian" % (shape, prec),
           rel_l2(host(out), oracle.fftnd_c2r(h.astype(np.complex128), shape[-1])), TOL[prec])
    np.testing.assert_array_equal(host(hd), h)
    p.close()


def _chunked_rel_l2(a, b_scaled_fn, rows=16):
    """rel-L2 of a against b = b_scaled_fn(i0 slice) over the leading axis in
    chunks (arrays of several GiB)."""
    num = den = 0.0
    for s in range(0, a.shape[0], rows):
        av = a[s:s + rows].astype(np.complex128)
        bv = b_scaled_fn(slice(s, s + rows))
        num += float(np.sum(np.abs(av - bv) ** 2))
        den += float(np.sum(np.abs(bv) ** 2))
    return (num / den) ** 0.5


def test_nd_4d_512x256x128x64_full_size():
    """The paper's 4-D C2C case, 512 x 256 x 128 x 64 complex64 (8 GiB),
    U[-1,1) seed 0, in the launch configuration the benchmark times: 16
    sampled outputs against the N-D definition, Parseval and the round trip
    over every element."""
    from paper_1506_07933_amd import Plan
    shape = (512, 256, 128, 64)
    x = synth.uniform_complex(shape, np.complex64, seed=0)
    p = Plan(shape, "c2c", "fp32")
    xd = gpu(x)
    yd = torch.empty_like(xd)
    p.forward(xd, out=yd)
    del xd
    Y = host(yd)
    rng = np.random.default_rng(54)
    ks = np.stack([rng.integers(0, n, 16) for n in shape], axis=1)
    ks[0] = 0  # the mean
    got = Y[tuple(ks.T)]
    report("4-D forward, 16 sampled outputs vs definition", rel_l2(got, dftnd_at(x, ks, -1)), 5e-6)
    n = float(x.size)
    ex = sum(float(np.sum(np.abs(x[s:s + 16].astype(np.complex128)) ** 2)) for s in range(0, 512, 16))
    ey = sum(float(np.sum(np.abs(Y[s:s + 16].astype(np.complex128)) ** 2)) for s in range(0, 512, 16))
    report("4-D Parseval |Y|^2 = N |x|^2", abs(ey / (n * ex) - 1.0), 5e-6)
    del Y
    p.inverse(yd, out=yd)
    Z = host(yd)
    del yd
    report("4-D round trip = N x", _chunked_rel_l2(Z, lambda sl: n * x[sl].astype(np.complex128)), 5e-6)
    p.close()
