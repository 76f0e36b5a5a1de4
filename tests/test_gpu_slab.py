"""GPU parity of the slab decomposition's local phases (Algorithm 3).

All p tasks of a slab-decomposed grid are held on the one GPU and the
all-to-all between the two halves is done with device copies; every task's
stages run through the C ABI.  The spectral shares are compared with the
oracle's slab transform (rel-L2 <= 1e-13 FP64, <= 5e-6 FP32, per share), the
inverse with the oracle's slab inverse of the same GPU shares, and the fused
stages (pack in the y-FFT's stores, unpack in the y-IFFT's loads) with the
standalone pack / unpack bit for bit.
"""
import numpy as np
import pytest

import oracle
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


def slab_forward(sp, x, fused=True, loopback=False):
    """Forward of all tasks: 2-D FFTs of each slab into its send buffer,
    exchange by device copies (task j receives block j of every sender, in
    sender order), x-FFT of each received slab."""
    p, n0l = sp.p, sp.n0l
    sends = []
    for r in range(p):
        a = x[r * n0l:(r + 1) * n0l].clone()  # a fresh buffer: the C ABI wants 16-byte alignment
        send = torch.empty(sp.send_shape, dtype=sp.cdtype, device=DEV)
        mid = torch.empty(sp.mid_shape, dtype=sp.cdtype, device=DEV)
        sp.forward_local(a, send, mid, fused=fused)
        sends.append(send)
    shares = []
    for j in range(p):
        recv = sends[0] if loopback else torch.stack([sends[s][j] for s in range(p)]).contiguous()
        out = torch.empty(sp.share_shape, dtype=sp.cdtype, device=DEV)
        sp.forward_x(recv, out)
        shares.append(out)
    return shares


def slab_inverse(sp, shares, fused=True, loopback=False):
    """Inverse of all tasks: x-IFFT of each share into its send buffer (block
    r = x rows of task r), exchange, unpack + y-IFFT + z-IFFT (C2R)."""
    p = sp.p
    sends = []
    for j in range(p):
        send = torch.empty(sp.send_shape, dtype=sp.cdtype, device=DEV)
        sp.inverse_x(shares[j], send)
        sends.append(send)
    outs = []
    for r in range(p):
        recv = sends[0] if loopback else torch.stack([sends[s][r] for s in range(p)]).contiguous()
        scratch = recv if loopback else torch.empty(sp.send_shape, dtype=sp.cdtype, device=DEV)
        out = torch.empty(sp.slab_shape, dtype=sp.sdtype, device=DEV)
        sp.inverse_local(recv, scratch, out, fused=fused)
        outs.append(out)
    return outs


C2C_CASES = [((64, 48, 40), 4, "fp32"), ((96, 60, 50), 3, "fp64"), ((32, 16, 8), 8, "fp32"),
             ((16, 8, 6), 8, "fp64"), ((128, 128, 128), 2, "fp32"), ((100, 120, 144), 4, "fp64"),
             ((27, 81, 25), 3, "fp32")]


@pytest.mark.parametrize("shape,p,prec", C2C_CASES)
def test_slab_c2c_all_tasks(shape, p, prec):
    from paper_1506_07933_amd import SlabPlan
    sp = SlabPlan(shape, p, "c2c", prec)
    x = synth.uniform_complex(shape, CDT[prec], seed=31)
    xd = gpu(x)
    shares = slab_forward(sp, xd, fused=True)
    ref = oracle.slab_forward(x.astype(np.complex128), p)
    for j in range(p):
        report("slab %s p=%d %s share %d" % (shape, p, prec, j), rel_l2(host(shares[j]), ref[j]), TOL[prec])
    unfused = slab_forward(sp, xd, fused=False)
    for j in range(p):
        assert torch.equal(shares[j], unfused[j]), "fused y+pack differs from y then pack"
    back = slab_inverse(sp, shares, fused=True)
    got = [host(b) for b in back]
    refi = oracle.slab_inverse([host(s).astype(np.complex128) for s in shares], p)
    for r in range(p):
        report("slab inverse task %d" % r, rel_l2(got[r], refi[r]), TOL[prec])
    report("slab round trip = N x", rel_l2(np.concatenate(got, axis=0), x.size * x.astype(np.complex128)),
           TOL[prec])
    back2 = slab_inverse(sp, shares, fused=False)
    for r in range(p):
        assert torch.equal(back[r], back2[r]), "fused unpack+y^-1 differs from unpack then y^-1"
    sp.close()


R2C_CASES = [((64, 48, 40), 4, "fp32"), ((60, 30, 18), 3, "fp64"), ((32, 16, 8), 8, "fp64"),
             ((128, 64, 256), 2, "fp32"), ((20, 20, 2), 4, "fp32")]


@pytest.mark.parametrize("shape,p,prec", R2C_CASES)
def test_slab_r2c_all_tasks(shape, p, prec):
    from paper_1506_07933_amd import SlabPlan
    sp = SlabPlan(shape, p, "r2c", prec)
    x = synth.normal_real(shape, RDT[prec], seed=32)
    shares = slab_forward(sp, gpu(x), fused=True)
    ref = oracle.slab_forward(x.astype(np.float64), p, real=True)
    for j in range(p):
        report("slab r2c %s p=%d %s share %d" % (shape, p, prec, j), rel_l2(host(shares[j]), ref[j]),
               TOL[prec])
    back = slab_inverse(sp, shares)
    report("slab r2c round trip = N x",
           rel_l2(np.concatenate([host(b) for b in back], axis=0), x.size * x.astype(np.float64)), TOL[prec])
    # a non-Hermitian spectrum: the C2R's discarded imaginary parts must not leak
    y = [synth.uniform_complex(sp.share_shape, CDT[prec], seed=40 + j) for j in range(p)]
    got = slab_inverse(sp, [gpu(v) for v in y], fused=False)
    refi = oracle.slab_inverse([v.astype(np.complex128) for v in y], p, n2=shape[2])
    for r in range(p):
        report("slab c2r non-Hermitian task %d" % r, rel_l2(host(got[r]), refi[r]), TOL[prec])
    sp.close()


@pytest.mark.parametrize("kind", ["c2c", "r2c"])
def test_slab_p1_loopback_is_the_full_transform(kind):
    """One task, receive buffer = send buffer: the slab stages are the whole
    3-D transform and match the oracle and the single-transform plan."""
    from paper_1506_07933_amd import Plan, SlabPlan
    shape = (48, 40, 64)
    sp = SlabPlan(shape, 1, kind, "fp64")
    if kind == "c2c":
        x = synth.uniform_complex(shape, np.complex128, seed=33)
        ref = oracle.fft3d_c2c(x, -1)
    else:
        x = synth.normal_real(shape, np.float64, seed=33)
        ref = oracle.fft3d_r2c(x)
    xd = gpu(x)
    (share,) = slab_forward(sp, xd, loopback=True)
    report("slab p=1 %s vs oracle" % kind, rel_l2(host(share), ref), 1e-13)
    pl = Plan(shape, kind, "fp64")
    report("slab p=1 %s vs Plan.forward" % kind, rel_l2(host(share), host(pl.forward(xd))), 1e-13)
    (back,) = slab_inverse(sp, [share], loopback=True)
    report("slab p=1 %s round trip" % kind, rel_l2(host(back), x.size * x), 1e-13)
    pl.close()
    sp.close()


def test_slab_stage_errors():
    from paper_1506_07933_amd import SlabPlan
    from paper_1506_07933_amd.fft import MifftError
    sp = SlabPlan((16, 16, 16), 4, "c2c", "fp32")
    a = torch.zeros(sp.slab_shape, dtype=torch.complex64, device=DEV)
    s = torch.zeros(sp.send_shape, dtype=torch.complex64, device=DEV)
    with pytest.raises(MifftError):        # pack is a forward stage only
        sp.stages(256 | 8, recv=s, send=s)
    with pytest.raises(MifftError):        # unpack in place across tasks
        sp.stages(256 | 16, recv=s, send=s)
    with pytest.raises(MifftError):        # z runs out of place
        sp.stages(1, src=a, out=a)
    with pytest.raises(MifftError):        # missing send buffer
        sp.stages(2 | 8, out=a)
    with pytest.raises(MifftError):        # empty mask
        sp.stages(0, src=a, out=s)
    sp.close()


def test_slab_512cube_four_tasks_full_size():
    """512^3 complex64 over 4 tasks, U[-1,1) seed 0, in the launch
    configuration the benchmark times: the stacked shares against the oracle's
    3-D DFT, and the round trip."""
    from paper_1506_07933_amd import SlabPlan
    shape, p = (512, 512, 512), 4
    sp = SlabPlan(shape, p, "c2c", "fp32")
    x = synth.uniform_complex(shape, np.complex64, seed=0)
    xd = gpu(x)
    shares = slab_forward(sp, xd)
    del xd
    ref = oracle.fft3d_c2c(x.astype(np.complex128), -1)
    n1l = sp.n1l
    for j in range(p):
        report("slab 512^3 p=4 share %d vs oracle" % j, rel_l2(host(shares[j]), ref[:, j * n1l:(j + 1) * n1l]),
               5e-6)
    del ref
    back = slab_inverse(sp, shares)
    del shares
    got = np.concatenate([host(b) for b in back], axis=0)
    report("slab 512^3 p=4 round trip", rel_l2(got, float(512 ** 3) * x.astype(np.complex128)), 5e-6)
    sp.close()
