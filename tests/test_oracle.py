"""Pins for the FP64 CPU oracle: it is checked against things fixed by the
mathematics, never against itself.

Each pin is chosen so a plausible mistake fails at least one test:
  * brute-force DFT on tiny grids (dropped terms, wrong twiddle, wrong radix)
  * the hand-derived 2x2x2 worked example in tests/golden
  * impulse -> constant, constant -> N delta, single mode -> N delta at m
    (index order / transposed axes), shift theorem (sign of the exponent)
  * Parseval, linearity, inverse(forward(x)) = N x (scaling convention)
  * Hermitian symmetry of R2C output and R2C = first half of C2C
  * numpy.fft (pocketfft) cross-check, including C2R on non-Hermitian input
  * the C2R definition written as an explicit cosine sum
  * the Poisson closed form for a sum of Fourier modes
  * the pencil pack / exchange / unpack maps against a textbook 2-D DFT
  * the slab decomposition (Algorithm 3) for all tasks against the brute
    force 3-D DFT, its inverse against the C2R cosine sum and N x
  * transforms of any rank against a direct N-D DFT sum over all index
    pairs, numpy.fft.fftn / rfftn / irfftn, and the 3-D oracle for a
    leading extent of 1
  * the spectral operators (Laplacian, Helmholtz, derivatives, gradient,
    divergence) against closed forms for sums of Fourier modes, the
    Nyquist-mode convention, and numpy's frequency grids
"""
import os

import numpy as np
import pytest

import oracle
from oracle.brute import brute_dft3, brute_dft3_at
from paper_1506_07933_amd import synth
from conftest import rel_l2

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def _rand_c(shape, seed):
    rng = np.random.default_rng(seed)
    return rng.uniform(-1, 1, shape) + 1j * rng.uniform(-1, 1, shape)


# ---------------------------------------------------------------- brute force

@pytest.mark.parametrize("shape", [(1, 1, 1), (1, 1, 7), (1, 1, 16), (2, 3, 5), (4, 4, 4),
                                   (6, 10, 15), (8, 12, 5), (7, 11, 13), (9, 25, 4),
                                   (16, 16, 16), (3, 49, 2)])
@pytest.mark.parametrize("sign", [-1, +1])
def test_brute_force_full(shape, sign):
    x = _rand_c(shape, seed=sum(shape))
    got = oracle.fft3d_c2c(x, sign)
    ref = brute_dft3(x, sign)
    assert rel_l2(got, ref) < 1e-12


@pytest.mark.parametrize("shape", [(32, 32, 32), (100, 12, 9), (5, 8, 125)])
def test_brute_force_sampled(shape):
    """32^3 and radix-5 heavy shapes, at 200 sampled outputs."""
    x = _rand_c(shape, seed=3)
    got = oracle.fft3d_c2c(x, -1)
    rng = np.random.default_rng(7)
    ks = np.stack([rng.integers(0, n, 200) for n in shape], axis=1)
    ks[0] = 0
    ref = brute_dft3_at(x, ks, -1)
    sel = got[ks[:, 0], ks[:, 1], ks[:, 2]]
    assert rel_l2(sel, ref) < 1e-12


def test_golden_2x2x2_by_hand():
    rows = np.loadtxt(os.path.join(GOLDEN, "dft_2x2x2_by_hand.txt"), comments="#")
    x = (np.arange(8, dtype=np.float64) + 1).reshape(2, 2, 2)
    got = oracle.fft3d_c2c(x, -1)
    for k0, k1, k2, re, im in rows:
        assert got[int(k0), int(k1), int(k2)] == pytest.approx(re + 1j * im, abs=1e-12)
    back = oracle.fft3d_c2c(got, +1)
    np.testing.assert_allclose(back.real, 8 * x, atol=1e-12)
    # the R2C / C2R pair on the same example
    half = oracle.fft3d_r2c(x)
    np.testing.assert_allclose(half, got[:, :, :2], atol=1e-12)
    np.testing.assert_allclose(oracle.fft3d_c2r(half, 2), 8 * x, atol=1e-12)


# ----------------------------------------------------------- closed forms

@pytest.mark.parametrize("shape", [(8, 12, 20), (5, 9, 16), (1, 1, 1)])
def test_impulse_and_constant(shape):
    n = int(np.prod(shape))
    d = np.zeros(shape, dtype=np.complex128)
    d[0, 0, 0] = 1.0
    np.testing.assert_allclose(oracle.fft3d_c2c(d, -1), np.ones(shape), atol=1e-13)
    one = np.ones(shape, dtype=np.complex128)
    expect = np.zeros(shape)
    expect[0, 0, 0] = n
    np.testing.assert_allclose(oracle.fft3d_c2c(one, -1), expect, atol=1e-11 * n)
    # R2C of the impulse is all ones; C2R of the all-ones half spectrum is N delta
    half = oracle.fft3d_r2c(d.real)
    np.testing.assert_allclose(half, np.ones(half.shape), atol=1e-13)
    back = oracle.fft3d_c2r(np.ones(half.shape, dtype=np.complex128), shape[2])
    np.testing.assert_allclose(back, expect, atol=1e-11 * n)


@pytest.mark.parametrize("m", [(1, 2, 3), (4, 0, 7), (5, 11, 19)])
def test_single_mode(m):
    """exp(+2 pi i m.x/n) transforms to N delta_{k,m}: pins index order."""
    shape = (6, 12, 20)
    a, b, c = np.meshgrid(*[np.arange(n) for n in shape], indexing="ij")
    ph = m[0] * a / shape[0] + m[1] * b / shape[1] + m[2] * c / shape[2]
    x = np.exp(2j * np.pi * ph)
    got = oracle.fft3d_c2c(x, -1)
    expect = np.zeros(shape, dtype=np.complex128)
    expect[m] = np.prod(shape)
    assert np.abs(got - expect).max() < 1e-10


def test_shift_theorem():
    """x shifted by s -> X * exp(-2 pi i k.s/n): pins the exponent's sign."""
    shape = (8, 10, 12)
    s = (3, 1, 5)
    x = _rand_c(shape, 11)
    xs = np.roll(x, s, axis=(0, 1, 2))
    kx = np.meshgrid(*[np.arange(n) for n in shape], indexing="ij")
    phase = np.exp(-2j * np.pi * sum(k * sh / n for k, sh, n in zip(kx, s, shape)))
    assert rel_l2(oracle.fft3d_c2c(xs, -1), oracle.fft3d_c2c(x, -1) * phase) < 1e-13
    # and the inverse has the opposite sign
    assert rel_l2(oracle.fft3d_c2c(xs, +1), oracle.fft3d_c2c(x, +1) / phase) < 1e-13


def test_cos_mode_two_spikes():
    n = (1, 1, 24)
    c = np.arange(24)
    x = np.cos(2 * np.pi * 5 * c / 24).reshape(n)
    got = oracle.fft3d_c2c(x, -1)[0, 0]
    expect = np.zeros(24)
    expect[5] = expect[19] = 12.0
    assert np.abs(got - expect).max() < 1e-12


@pytest.mark.parametrize("n", [2, 3, 4, 5, 7, 8, 12, 30, 64])
def test_one_dimensional_reduction(n):
    """n0 = n1 = 1 is the 1-D DFT, X[k] = sum_j x[j] exp(-2 pi i jk/n)."""
    x = _rand_c((1, 1, n), n)
    j = np.arange(n)
    mat = np.exp(-2j * np.pi * np.outer(j, j) / n)
    assert rel_l2(oracle.fft3d_c2c(x, -1)[0, 0], mat @ x[0, 0]) < 1e-13


# -------------------------------------------------------------- invariants

@pytest.mark.parametrize("shape", [(12, 18, 10), (32, 32, 32), (16, 24, 125)])
def test_parseval_roundtrip_linearity(shape):
    n = int(np.prod(shape))
    x = _rand_c(shape, 1)
    y = _rand_c(shape, 2)
    fx = oracle.fft3d_c2c(x, -1)
    fy = oracle.fft3d_c2c(y, -1)
    assert abs(np.sum(np.abs(fx) ** 2) / (n * np.sum(np.abs(x) ** 2)) - 1) < 1e-12
    assert rel_l2(oracle.fft3d_c2c(fx, +1), n * x) < 1e-13
    al, be = 0.3 - 1.2j, 2.5 + 0.1j
    assert rel_l2(oracle.fft3d_c2c(al * x + be * y, -1), al * fx + be * fy) < 1e-13


@pytest.mark.parametrize("shape", [(6, 8, 10), (5, 7, 9), (16, 16, 32), (4, 6, 1)])
def test_r2c_hermitian_and_half(shape):
    rng = np.random.default_rng(5)
    x = rng.standard_normal(shape)
    half = oracle.fft3d_r2c(x)
    n0, n1, n2 = shape
    assert half.shape == (n0, n1, n2 // 2 + 1)
    # k2 = 0 plane (and k2 = n2/2 for even n2) is Hermitian in (k0, k1)
    planes = [0] + ([n2 // 2] if n2 % 2 == 0 else [])
    i0 = (-np.arange(n0)) % n0
    i1 = (-np.arange(n1)) % n1
    for p in planes:
        pl = half[:, :, p]
        assert np.abs(pl - np.conj(pl[i0][:, i1])).max() < 1e-12
    full = oracle.fft3d_c2c(x.astype(np.complex128), -1)
    assert rel_l2(half, full[:, :, : n2 // 2 + 1]) < 1e-14
    # every entry of the full spectrum is the conjugate of its mirror
    k2 = (-np.arange(n2)) % n2
    assert np.abs(full - np.conj(full[i0][:, i1][:, :, k2])).max() < 1e-12


# ---------------------------------------------------------- library check

@pytest.mark.parametrize("shape", [(32, 32, 32), (48, 64, 96), (100, 120, 144),
                                   (125, 25, 5), (3, 384, 8), (1, 1, 1024), (7, 13, 6)])
def test_numpy_cross_check_c2c(shape):
    x = _rand_c(shape, 9)
    assert rel_l2(oracle.fft3d_c2c(x, -1), np.fft.fftn(x)) < 1e-13
    n = int(np.prod(shape))
    assert rel_l2(oracle.fft3d_c2c(x, +1), n * np.fft.ifftn(x)) < 1e-13


@pytest.mark.parametrize("shape", [(16, 16, 16), (64, 32, 48), (20, 30, 100), (5, 6, 7),
                                   (8, 8, 1), (4, 4, 2)])
def test_numpy_cross_check_real(shape):
    rng = np.random.default_rng(21)
    x = rng.standard_normal(shape)
    half = oracle.fft3d_r2c(x)
    assert rel_l2(half, np.fft.rfftn(x, axes=(0, 1, 2))) < 1e-13
    n = int(np.prod(shape))
    # non-Hermitian half spectrum: imaginary parts at k2 = 0 and n2/2 matter
    y = rng.standard_normal(half.shape) + 1j * rng.standard_normal(half.shape)
    ref = n * np.fft.irfftn(y, s=shape, axes=(0, 1, 2))
    assert rel_l2(oracle.fft3d_c2r(y, shape[2]), ref) < 1e-13
    # round trip
    assert rel_l2(oracle.fft3d_c2r(half, shape[2]), n * x) < 1e-13


def test_c2r_explicit_cosine_sum():
    """C2R along z written as x[c] = Re Y0 + (-1)^c Re Y[n/2]
    + 2 sum_{k=1}^{n/2-1} Re(Y[k] exp(+2 pi i k c/n)) after inverse DFTs along
    x and y done with explicit matrices (even and odd n2)."""
    rng = np.random.default_rng(4)
    for shape in [(3, 4, 8), (5, 2, 9), (2, 3, 2), (4, 4, 1)]:
        n0, n1, n2 = shape
        h = n2 // 2 + 1
        y = rng.standard_normal((n0, n1, h)) + 1j * rng.standard_normal((n0, n1, h))
        m0 = np.exp(2j * np.pi * np.outer(np.arange(n0), np.arange(n0)) / n0)
        m1 = np.exp(2j * np.pi * np.outer(np.arange(n1), np.arange(n1)) / n1)
        t = np.einsum("ak,kbz->abz", m0, y)
        t = np.einsum("bk,akz->abz", m1, t)
        c = np.arange(n2)
        out = np.repeat(t[:, :, :1].real, n2, axis=2)
        top = (n2 - 1) // 2
        for k in range(1, top + 1):
            out += 2 * np.real(t[:, :, k:k + 1] * np.exp(2j * np.pi * k * c / n2))
        if n2 % 2 == 0 and n2 > 1:
            out += t[:, :, n2 // 2:n2 // 2 + 1].real * ((-1.0) ** c)
        assert rel_l2(oracle.fft3d_c2r(y, n2), out) < 1e-13


# ----------------------------------------------------------------- Poisson

@pytest.mark.parametrize("n", [16, 24, 32])
def test_poisson_closed_form(n):
    """f = sum a_j cos(k_j.x + phi_j) -> u = -sum a_j cos(k_j.x + phi_j)/|k_j|^2."""
    ks, amp, phase, _ = synth.poisson_modes(n, seed=n)
    f = synth.mode_sum(n, ks, amp, phase)
    u = oracle.poisson_solve(f)
    ref = synth.mode_sum(n, ks, -amp / np.sum(ks * ks, axis=1), phase)
    assert rel_l2(u, ref) < 1e-12


def test_poisson_kills_mean_and_matches_numpy():
    n = 16
    rng = np.random.default_rng(3)
    f = rng.standard_normal((n, n, n)) + 5.0
    u = oracle.poisson_solve(f)
    assert abs(u.mean()) < 1e-14
    k = np.fft.fftfreq(n, 1.0 / n)
    kk = k[:, None, None] ** 2 + k[None, :, None] ** 2 + np.fft.rfftfreq(n, 1.0 / n)[None, None, :] ** 2
    kk[0, 0, 0] = np.inf
    ref = np.fft.irfftn(-np.fft.rfftn(f) / kk, s=f.shape, axes=(0, 1, 2))
    assert rel_l2(u, ref) < 1e-13


# ------------------------------------------------------------ pencil maps

def test_pack_unpack_are_permutations():
    a = np.arange(4 * 6 * 8).reshape(4, 6, 8)
    s = oracle.pencil_pack(a, 4)
    assert s.shape == (4, 4, 6, 2)
    for j in range(4):
        np.testing.assert_array_equal(s[j], a[:, :, 2 * j:2 * j + 2])
    b = oracle.pencil_unpack(s, 6)
    assert b.shape == (4, 24, 2)
    for j in range(4):
        np.testing.assert_array_equal(b[:, 6 * j:6 * j + 6, :], s[j])
    assert sorted(b.ravel().tolist()) == list(range(a.size))


def test_pencil_share_loopback():
    """Loopback share = z-DFT, pack, identity exchange, unpack, y-DFT; checked
    with numpy FFTs applied to the explicitly permuted array."""
    a = _rand_c((3, 4, 8), 12)
    got = oracle.pencil_share_forward(a, 2)
    ahat = np.fft.fft(a, axis=2)
    b = np.concatenate([ahat[:, :, 0:4], ahat[:, :, 4:8]], axis=1)
    assert rel_l2(got, np.fft.fft(b, axis=1)) < 1e-13


def test_pencil_row_group_emulation():
    """With all p1 ranks of a row held at once and a true all-to-all, rank j's
    block after the y-DFT is the k2 slice j of the 2-D (y, z) DFT of the slab."""
    p1, n0l, n1l, n2 = 4, 2, 3, 8
    g = _rand_c((n0l, p1 * n1l, n2), 8)
    shares = [g[:, r * n1l:(r + 1) * n1l, :] for r in range(p1)]
    sends = [oracle.pencil_pack(oracle.fft_axis(s, 2, -1), p1) for s in shares]
    m = n2 // p1
    # textbook 2-D (y, z) DFT of each x-slab: a brute-force 3-D DFT with n0 = 1
    ref = np.stack([brute_dft3(g[i][None], -1)[0] for i in range(n0l)])
    for j in range(p1):
        recv = np.stack([sends[r][j] for r in range(p1)])
        b = oracle.pencil_unpack(recv, n1l)
        got = oracle.fft_axis(b, 1, -1)
        assert rel_l2(got, ref[:, :, j * m:(j + 1) * m]) < 1e-13


# ------------------------------------------------- other spectral operators

def _modes(n, seed):
    ks, amp, phase, _ = synth.poisson_modes(n, seed=seed)
    return ks, amp, phase


@pytest.mark.parametrize("n", [16, 24])
def test_laplacian_and_helmholtz_closed_form(n):
    """lap cos(k.x + p) = -|k|^2 cos(k.x + p); (alpha - lap) u = f for
    u = cos(k.x + p) / (alpha + |k|^2)."""
    ks, amp, phase = _modes(n, 40 + n)
    f = synth.mode_sum(n, ks, amp, phase)
    kk = np.sum(ks * ks, axis=1).astype(np.float64)
    lap = oracle.spectral_apply(f, oracle.OP_LAPLACIAN)
    assert rel_l2(lap, synth.mode_sum(n, ks, -amp * kk, phase)) < 1e-12
    for alpha in (0.5, 3.0):
        u = oracle.spectral_apply(f, oracle.OP_HELMHOLTZ, alpha)
        assert rel_l2(u, synth.mode_sum(n, ks, amp / (alpha + kk), phase)) < 1e-12
    # alpha = 0 is the Poisson solve with the opposite sign
    assert rel_l2(oracle.spectral_apply(f, oracle.OP_HELMHOLTZ, 0.0), -oracle.poisson_solve(f)) < 1e-13


@pytest.mark.parametrize("n", [16, 18])
def test_gradient_and_divergence_closed_form(n):
    """d/dx_j cos(k.x + p) = k_j cos(k.x + p + pi/2), for modes below the
    Nyquist index; the divergence of three mode sums is the sum of those."""
    ks, amp, phase = _modes(n, 50 + n)
    f = synth.mode_sum(n, ks, amp, phase)
    g = oracle.gradient(f)
    for j in range(3):
        ref = synth.mode_sum(n, ks, amp * ks[:, j], phase + np.pi / 2)
        assert rel_l2(g[j], ref) < 1e-12
    rng = np.random.default_rng(n)
    amps = [rng.standard_normal(len(ks)) for _ in range(3)]
    v = [synth.mode_sum(n, ks, a, phase) for a in amps]
    d = oracle.divergence(*v)
    ref = sum(synth.mode_sum(n, ks, a * ks[:, j], phase + np.pi / 2) for j, a in enumerate(amps))
    assert rel_l2(d, ref) < 1e-12
    # the divergence of a gradient is the Laplacian (no Nyquist content here)
    assert rel_l2(oracle.divergence(*g), oracle.spectral_apply(f, oracle.OP_LAPLACIAN)) < 1e-12


def test_derivative_nyquist_mode_is_zero():
    """On an even grid the highest mode cos(n x / 2) = (-1)^i has no
    well-defined derivative sign; the convention sets it to zero.  Odd grids
    have no such mode and differentiate every mode."""
    n = 8
    i = np.arange(n)
    f = np.broadcast_to(((-1.0) ** i)[:, None, None], (n, n, n)).copy()
    for op in (oracle.OP_DX, oracle.OP_DY, oracle.OP_DZ):
        assert np.max(np.abs(oracle.spectral_apply(np.moveaxis(f, 0, op - oracle.OP_DX), op))) < 1e-13
    m = oracle.spectral_multiplier((6, 5, 8), oracle.OP_DX)
    assert np.all(m[3] == 0) and np.all(m[2] == 2j) and np.all(m[4] == -2j)
    m = oracle.spectral_multiplier((6, 5, 8), oracle.OP_DY)
    assert np.all(m[:, 2] == 2j) and np.all(m[:, 3] == -2j)      # n1 = 5: no Nyquist index
    m = oracle.spectral_multiplier((6, 5, 8), oracle.OP_DZ)
    assert np.all(m[..., 4] == 0) and np.all(m[..., 3] == 3j)


def test_spectral_multipliers_match_numpy_frequencies():
    shape = (6, 10, 12)
    k0 = np.fft.fftfreq(6, 1 / 6)[:, None, None]
    k1 = np.fft.fftfreq(10, 1 / 10)[None, :, None]
    k2 = np.fft.rfftfreq(12, 1 / 12)[None, None, :]
    kk = k0 ** 2 + k1 ** 2 + k2 ** 2
    np.testing.assert_allclose(oracle.spectral_multiplier(shape, oracle.OP_LAPLACIAN), np.broadcast_to(-kk, (6, 10, 7)))
    p = oracle.spectral_multiplier(shape, oracle.OP_POISSON)
    assert p[0, 0, 0] == 0
    np.testing.assert_allclose(p.ravel()[1:], -1 / kk.ravel()[1:])
    # the Poisson multiplier agrees with the C oracle's multiply
    y = _rand_c((6, 10, 7), 60)
    np.testing.assert_allclose(y * p, oracle.poisson_half(y, 12), rtol=1e-14, atol=1e-15)


# -------------------------------------------------------------- slab maps

def test_slab_pack_is_the_y_split():
    a = np.arange(3 * 8 * 5).reshape(3, 8, 5)
    s = oracle.slab_pack(a, 4)
    assert s.shape == (4, 3, 2, 5)
    for j in range(4):
        np.testing.assert_array_equal(s[j], a[:, 2 * j:2 * j + 2, :])
    assert sorted(s.ravel().tolist()) == list(range(a.size))


@pytest.mark.parametrize("shape,p", [((4, 6, 5), 2), ((6, 6, 4), 3), ((8, 4, 3), 4),
                                     ((2, 2, 7), 1), ((4, 8, 1), 4)])
def test_slab_forward_c2c_brute(shape, p):
    """Shares stacked along y are the full 3-D DFT (brute force): a wrong pack
    order, a wrong receive order or a missing x-DFT all fail here."""
    x = _rand_c(shape, 21)
    shares = oracle.slab_forward(x, p)
    n1l = shape[1] // p
    assert all(s.shape == (shape[0], n1l, shape[2]) for s in shares)
    assert rel_l2(np.concatenate(shares, axis=1), brute_dft3(x, -1)) < 1e-13


@pytest.mark.parametrize("shape,p", [((4, 6, 6), 2), ((6, 3, 5), 3), ((4, 4, 2), 4)])
def test_slab_forward_r2c_brute(shape, p):
    rng = np.random.default_rng(22)
    x = rng.standard_normal(shape)
    shares = oracle.slab_forward(x, p, real=True)
    ref = brute_dft3(x.astype(np.complex128), -1)[..., :shape[2] // 2 + 1]
    assert rel_l2(np.concatenate(shares, axis=1), ref) < 1e-13


@pytest.mark.parametrize("shape,p", [((4, 6, 5), 2), ((6, 6, 8), 3), ((4, 4, 4), 4)])
def test_slab_inverse_roundtrip(shape, p):
    x = _rand_c(shape, 23)
    back = oracle.slab_inverse(oracle.slab_forward(x, p), p)
    assert all(b.shape == (shape[0] // p,) + shape[1:] for b in back)
    assert rel_l2(np.concatenate(back, axis=0), x.size * x) < 1e-13


def test_slab_inverse_c2r_cosine_sum():
    """Non-Hermitian half spectrum through the slab inverse: x- and y-IDFTs as
    explicit matrices, then the C2R cosine sum (odd and even n2)."""
    rng = np.random.default_rng(24)
    for (n0, n1, n2), p in [((4, 6, 8), 2), ((6, 3, 7), 3), ((4, 4, 2), 4)]:
        h = n2 // 2 + 1
        y = rng.standard_normal((n0, n1, h)) + 1j * rng.standard_normal((n0, n1, h))
        n1l = n1 // p
        shares = [y[:, j * n1l:(j + 1) * n1l, :] for j in range(p)]
        got = np.concatenate(oracle.slab_inverse(shares, p, n2=n2), axis=0)
        m0 = np.exp(2j * np.pi * np.outer(np.arange(n0), np.arange(n0)) / n0)
        m1 = np.exp(2j * np.pi * np.outer(np.arange(n1), np.arange(n1)) / n1)
        t = np.einsum("bk,akz->abz", m1, np.einsum("ak,kbz->abz", m0, y))
        c = np.arange(n2)
        ref = np.repeat(t[:, :, :1].real, n2, axis=2)
        for k in range(1, (n2 - 1) // 2 + 1):
            ref += 2 * np.real(t[:, :, k:k + 1] * np.exp(2j * np.pi * k * c / n2))
        if n2 % 2 == 0 and n2 > 1:
            ref += t[:, :, n2 // 2:n2 // 2 + 1].real * ((-1.0) ** c)
        assert rel_l2(got, ref) < 1e-13


def test_c2r_z_lines():
    """The z-only C2R: round trip of real lines (n2 x), and the imaginary parts
    at k = 0 and k = n2/2 have no effect."""
    rng = np.random.default_rng(25)
    for n2 in (1, 2, 7, 8, 30):
        x = rng.standard_normal((3, 4, n2))
        half = np.fft.fft(x, axis=2)[..., :n2 // 2 + 1]
        assert rel_l2(oracle.c2r_z(half, n2), n2 * x) < 1e-13
        bent = half.copy()
        bent[..., 0] += 3j
        if n2 % 2 == 0:
            bent[..., n2 // 2] -= 2j
        np.testing.assert_array_equal(oracle.c2r_z(bent, n2), oracle.c2r_z(half, n2))


# ------------------------------------------------------------ any rank

def _direct_dft_nd(x, sign):
    """X[k] = sum_a x[a] exp(sign 2 pi i sum_j k_j a_j / n_j), every (k, a) pair
    at once: one dense matrix over all flattened index pairs (tiny arrays)."""
    shape = x.shape
    idx = np.stack(np.unravel_index(np.arange(x.size), shape), axis=1).astype(np.float64)
    frac = idx / np.asarray(shape, dtype=np.float64)
    phase = (idx @ frac.T) % 1.0           # sum_j k_j a_j / n_j for every (k, a)
    return (np.exp(sign * 2j * np.pi * phase) @ x.ravel()).reshape(shape)


@pytest.mark.parametrize("shape", [(2, 3, 4, 5), (4, 1, 6, 2), (3, 2, 2, 2, 3), (5,), (6, 10),
                                   (1, 1, 1, 1), (2, 2, 3, 1, 2, 2)])
@pytest.mark.parametrize("sign", [-1, +1])
def test_fftnd_direct_sum(shape, sign):
    x = _rand_c(shape, 26)
    assert rel_l2(oracle.fftnd_c2c(x, sign), _direct_dft_nd(x, sign)) < 1e-13


def test_dftnd_at_sampled_definition():
    """The sampled N-D definition (used where the full oracle is too large)
    against the dense direct sum on tiny arrays, and against the FFT oracle
    at random outputs of a 4-D array."""
    from oracle.brute import dftnd_at
    for shape in [(2, 3, 4, 5), (3, 1, 2, 2, 4), (7,)]:
        x = _rand_c(shape, 31)
        allk = np.stack(np.unravel_index(np.arange(x.size), shape), axis=1)
        for sign in (-1, 1):
            got = dftnd_at(x, allk, sign, chunk_rows=3).reshape(shape)
            assert rel_l2(got, _direct_dft_nd(x, sign)) < 1e-13
    x = _rand_c((8, 6, 10, 12), 32)
    rng = np.random.default_rng(33)
    ks = np.stack([rng.integers(0, n, 20) for n in x.shape], axis=1)
    ref = oracle.fftnd_c2c(x, -1)[tuple(ks.T)]
    assert rel_l2(dftnd_at(x.astype(np.complex64), ks, -1), oracle.fftnd_c2c(x.astype(np.complex64), -1)[tuple(ks.T)]) < 1e-13
    assert rel_l2(dftnd_at(x, ks, -1, chunk_rows=7), ref) < 1e-13


def test_fftnd_matches_numpy_and_3d():
    x = _rand_c((4, 6, 10, 8), 27)
    assert rel_l2(oracle.fftnd_c2c(x, -1), np.fft.fftn(x)) < 1e-13
    assert rel_l2(oracle.fftnd_c2c(x, +1), x.size * np.fft.ifftn(x)) < 1e-13
    y = _rand_c((1, 6, 10, 8), 28)
    assert rel_l2(oracle.fftnd_c2c(y, -1)[0], oracle.fft3d_c2c(y[0], -1)) < 1e-13
    rng = np.random.default_rng(29)
    r = rng.standard_normal((3, 5, 4, 6))
    assert rel_l2(oracle.fftnd_r2c(r), np.fft.rfftn(r)) < 1e-13
    h = _rand_c((3, 5, 4, 4), 30)      # not Hermitian: numpy drops the same parts
    n = 3 * 5 * 4 * 6
    assert rel_l2(oracle.fftnd_c2r(h, 6), n * np.fft.irfftn(h, s=(3, 5, 4, 6), axes=(0, 1, 2, 3))) < 1e-13
    assert rel_l2(oracle.fftnd_c2r(oracle.fftnd_r2c(r), 6), r.size * r) < 1e-13


def test_fft_axis_matches_numpy():
    x = _rand_c((3, 5, 7, 4), 2)
    for ax in range(4):
        assert rel_l2(oracle.fft_axis(x, ax, -1), np.fft.fft(x, axis=ax)) < 1e-13


def test_unit_root_quarter_turns_exact():
    """Multiples of a quarter turn come out exact (0, +-1)."""
    for n in (4, 8, 12, 100, 1024):
        x = np.zeros((1, 1, n), dtype=np.complex128)
        x[0, 0, 1] = 1.0
        row = oracle.fft3d_c2c(x, -1)[0, 0]   # row[k] = exp(-2 pi i k/n)
        for k, expect in ((0, 1), (n // 4, -1j), (n // 2, -1), (3 * n // 4, 1j)):
            assert row[k] == expect
