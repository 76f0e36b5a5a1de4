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
