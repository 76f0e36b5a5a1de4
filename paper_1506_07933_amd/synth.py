"""Seeded synthetic inputs for the 3-D FFT workloads.

This module is the only code shared by the HIP path's tests and the CPU
oracle's tests: it draws random numbers and lays them out, and holds none of
the transform's arithmetic.  The paper measures on synthetic grids whose
values it never describes (Sec. 3, "Parameters in the Experiments"), so every
workload here is seeded and synthetic.

Recipes (numpy ``default_rng(seed)``; real parts are drawn first, then
imaginary parts, each as one C-order array; float32 data are the float64
draws rounded to nearest):

* ``uniform_complex``  re, im ~ U[-1, 1)            (32^3 c128, 512^3 c64,
                                                    the 256x256x1024 share)
* ``normal_real``      x ~ N(0, 1)                  (256^3 R2C/C2R)
* ``normal_complex``   re, im ~ N(0, 1)             (batched uneven sizes)
* ``batched_uneven``   64 shapes drawn with ``rng.choice`` from the six sizes,
                       then each transform's re, im from the same generator
* ``poisson_rhs``      8 random Fourier modes plus N(0, 0.01) noise; the
                       modes are returned too so a closed form can be checked
* ``arrival_schedule`` exponential inter-arrival times at a given rate, grid
                       size uniform over the five sizes, float32 w.p. 0.8
* ``poisson_rhs_device`` the Poisson right-hand side recipe written into a
                       caller's device array (the served requests draw theirs
                       this way, one seed per request)
"""
from __future__ import annotations

import math

import numpy as np

UNEVEN_SHAPES = ((48, 48, 48), (64, 64, 64), (96, 96, 96), (128, 128, 128),
                 (100, 120, 144), (125, 125, 125))
SERVE_SIZES = (64, 128, 256, 384, 512)


def _cast_complex(re: np.ndarray, im: np.ndarray, dtype) -> np.ndarray:
    dtype = np.dtype(dtype)
    if dtype == np.complex64:
        out = np.empty(re.shape, dtype=np.complex64)
        out.real = re.astype(np.float32)
        out.imag = im.astype(np.float32)
        return out
    if dtype == np.complex128:
        out = np.empty(re.shape, dtype=np.complex128)
        out.real = re
        out.imag = im
        return out
    raise ValueError("complex dtype expected, got %s" % dtype)


def uniform_complex(shape, dtype=np.complex64, seed: int = 0) -> np.ndarray:
    rng = np.random.default_rng(seed)
    re = rng.uniform(-1.0, 1.0, size=shape)
    im = rng.uniform(-1.0, 1.0, size=shape)
    return _cast_complex(re, im, dtype)


def normal_complex(shape, dtype=np.complex64, seed: int = 0, rng=None) -> np.ndarray:
    rng = np.random.default_rng(seed) if rng is None else rng
    re = rng.standard_normal(size=shape)
    im = rng.standard_normal(size=shape)
    return _cast_complex(re, im, dtype)


def normal_real(shape, dtype=np.float64, seed: int = 0) -> np.ndarray:
    rng = np.random.default_rng(seed)
    return rng.standard_normal(size=shape).astype(dtype)


def batched_uneven(count: int = 64, seed: int = 0, dtype=np.complex64, shapes=UNEVEN_SHAPES):
    """Shapes drawn with ``rng.choice`` over ``shapes`` (count draws), then one
    N(0,1) complex array per transform, in order, from the same generator."""
    rng = np.random.default_rng(seed)
    idx = rng.choice(len(shapes), size=count)
    dims = [tuple(shapes[i]) for i in idx]
    data = [normal_complex(d, dtype=dtype, rng=rng) for d in dims]
    return dims, data


def poisson_modes(n: int, seed: int, count: int = 8):
    """``count`` random Fourier modes for an n^3 periodic grid: integer wave
    vectors with components uniform in [-K, K], K = min(8, n/2 - 1), k != 0;
    amplitudes N(0, 1); phases U[0, 2 pi)."""
    rng = np.random.default_rng(seed)
    kmax = min(8, n // 2 - 1)
    ks = []
    while len(ks) < count:
        k = rng.integers(-kmax, kmax + 1, size=3)
        if np.any(k != 0):
            ks.append(k)
    ks = np.array(ks, dtype=np.int64)
    amp = rng.standard_normal(size=count)
    phase = rng.uniform(0.0, 2.0 * np.pi, size=count)
    return ks, amp, phase, rng


def mode_sum(n: int, ks, amp, phase) -> np.ndarray:
    """sum_j amp_j cos(k_j . x + phase_j) on the grid x_i = 2 pi i / n, built
    from per-axis angles so no n^3 temporary per mode is complex."""
    x = 2.0 * np.pi * np.arange(n, dtype=np.float64) / n
    out = np.zeros((n, n, n), dtype=np.float64)
    for k, a, p in zip(ks, amp, phase):
        ab = k[0] * x[:, None] + k[1] * x[None, :] + p
        cab, sab = np.cos(ab), np.sin(ab)
        c = k[2] * x
        cc, sc = np.cos(c), np.sin(c)
        out += a * (cab[:, :, None] * cc[None, None, :] - sab[:, :, None] * sc[None, None, :])
    return out


def poisson_rhs(n: int, seed: int, dtype=np.float64, noise: float = 0.01):
    """Right-hand side = 8 random modes + N(0, noise^2) white noise.
    Returns (rhs, (ks, amp, phase)); float32 data are rounded float64 draws."""
    ks, amp, phase, rng = poisson_modes(n, seed)
    f = mode_sum(n, ks, amp, phase)
    if noise:
        f += noise * rng.standard_normal(size=f.shape)
    return f.astype(dtype), (ks, amp, phase)


def arrival_schedule(count: int, rate: float, seed: int = 0, sizes=SERVE_SIZES,
                     fp32_fraction: float = 0.8):
    """Open-loop request stream: arrival times (s), grid size, precision."""
    rng = np.random.default_rng(seed)
    gaps = rng.exponential(1.0 / rate, size=count)
    t = np.cumsum(gaps) - gaps[0]
    n = rng.choice(np.asarray(sizes), size=count)
    fp32 = rng.random(size=count) < fp32_fraction
    return [(float(t[i]), int(n[i]), "fp32" if fp32[i] else "fp64") for i in range(count)]


def poisson_rhs_torch(n: int, seed: int, dtype, device, noise: float = 0.01):
    """The Poisson right-hand side recipe evaluated on the device: the same 8
    seeded modes as ``poisson_modes``, summed in float64, plus N(0, noise^2)
    noise from a torch generator seeded with ``seed``; cast to ``dtype``.
    Used where host generation of large grids would stall the caller; the
    values are copied back whenever a CPU check needs them."""
    import torch
    ks, amp, phase, _ = poisson_modes(n, seed)
    x = 2.0 * math.pi * torch.arange(n, dtype=torch.float64, device=device) / n
    out = torch.zeros((n, n, n), dtype=torch.float64, device=device)
    for k, a, p in zip(ks, amp, phase):
        ab = float(k[0]) * x[:, None] + float(k[1]) * x[None, :] + float(p)
        c = float(k[2]) * x
        out += float(a) * (torch.cos(ab)[:, :, None] * torch.cos(c)[None, None, :]
                           - torch.sin(ab)[:, :, None] * torch.sin(c)[None, None, :])
    if noise:
        g = torch.Generator(device=device)
        g.manual_seed(int(seed))
        out += noise * torch.randn((n, n, n), generator=g, dtype=torch.float64, device=device)
    return out.to(dtype)


def poisson_rhs_device(out, seed: int, noise: float = 0.01, stream=None, staging=None):
    """The Poisson right-hand side recipe written into the device array
    ``out`` (n x n x n, float32 or float64) on ``stream``: the 8 modes of
    ``poisson_modes(n, seed)`` plus N(0, noise^2) noise from a torch device
    generator seeded with ``seed`` (``mode_sum_device``).  The values depend
    only on (n, seed, dtype)."""
    ks, amp, phase, _ = poisson_modes(out.shape[0], seed)
    return mode_sum_device(out, ks, amp, phase, noise=noise, seed=seed, stream=stream, staging=staging)


def mode_sum_device(out, ks, amp, phase, noise: float = 0.0, seed: int = 0, stream=None, staging=None):
    """sum_j amp_j cos(k_j . x + phase_j) (the ``mode_sum`` grid) plus
    N(0, noise^2) noise, written into the device array ``out`` (n x n x n,
    float32 or float64) on ``stream``.  The sum is separable,
    cos(a + b + c) = Re(e^{ia} e^{ib} e^{ic}), so it is evaluated as one
    matrix product: out[(x, y), z] += sum_j Re(A_j[x, y] E_j[z]) with
    A_j = amp_j e^{i phase_j} e^{i kx_j x} e^{i ky_j y} and E_j = e^{i kz_j z}
    (real and imaginary parts as a rank-2J product), after the noise (from a
    torch device generator seeded with ``seed``) is drawn into ``out``.  The
    per-axis factors are built on the host in float64 and copied in (through
    ``staging``, a pinned complex128 host tensor of at least 3 J n elements,
    when given, so the copy does not block the caller; it must not be reused
    before this stream's work is done)."""
    import torch
    n = out.shape[0]
    ks = np.asarray(ks, dtype=np.int64)
    amp = np.asarray(amp, dtype=np.float64)
    phase = np.asarray(phase, dtype=np.float64)
    J = len(amp)
    x = 2.0 * np.pi * np.arange(n, dtype=np.float64) / n
    ex = np.exp(1j * (ks[:, 0:1] * x[None, :] + phase[:, None])) * amp[:, None]   # (J, n)
    ey = np.exp(1j * ks[:, 1:2] * x[None, :])                                      # (J, n)
    ez = np.exp(1j * ks[:, 2:3] * x[None, :])                                      # (J, n)
    dt = out.dtype
    s = torch.cuda.current_stream(out.device) if stream is None else stream
    with torch.cuda.stream(s):
        host = np.stack([ex, ey, ez])
        if staging is not None:
            st = staging[:3 * J * n].view(3, J, n)
            st.copy_(torch.from_numpy(host))
            tab = st.to(out.device, non_blocking=True)
        else:
            tab = torch.from_numpy(host).to(out.device)
        a = tab[0][:, :, None] * tab[1][:, None, :]                                # (J, n, n)
        lhs = torch.cat([a.real, -a.imag]).reshape(2 * J, n * n).to(dt)            # (2J, n^2)
        rhs = torch.cat([tab[2].real, tab[2].imag]).to(dt)                         # (2J, n)
        f2 = out.view(n * n, n)
        if noise:
            g = torch.Generator(device=out.device)
            g.manual_seed(int(seed))
            f2.normal_(0.0, noise, generator=g)
        else:
            f2.zero_()
        f2.addmm_(lhs.t(), rhs)
    return out
