"""Direct O(N^2) 3-D DFT: the definition, summed term by term (and the N-D
definition at sampled outputs, ``dftnd_at``).

TEST INFRASTRUCTURE ONLY (pins the oracle; see the package docstring).

X[k0,k1,k2] = sum_{a,b,c} x[a,b,c] exp(sign 2 pi i (k0 a/n0 + k1 b/n1 + k2 c/n2))
(the discrete 3-D Fourier transform the paper calls a dense matrix-vector
product, Sec. 2).  The phase of every term is reduced exactly in integers:
with L = lcm(n0, n1, n2) the phase is 2 pi e / L where
e = (k0 a L/n0 + k1 b L/n1 + k2 c L/n2) mod L, and exp(2 pi i e / L) is read
from one table of the L-th roots of unity.  The sum over inputs is a dense
matrix-vector product computed in row chunks, so memory stays bounded; it
shares nothing with the Cooley-Tukey code it pins.
"""
from __future__ import annotations

import math

import numpy as np


def _lcm(a: int, b: int) -> int:
    return a * b // math.gcd(a, b)


def brute_dft3(x, sign: int = -1, chunk_elems: int = 1 << 23) -> np.ndarray:
    x = np.asarray(x, dtype=np.complex128)
    if x.ndim != 3:
        raise ValueError("brute_dft3 needs a 3-D array")
    n0, n1, n2 = x.shape
    big_l = _lcm(_lcm(n0, n1), n2)
    table = np.exp(sign * 2j * np.pi * np.arange(big_l, dtype=np.float64) / big_l)
    a, b, c = np.meshgrid(np.arange(n0), np.arange(n1), np.arange(n2), indexing="ij")
    # per-input phase step for each output axis, in units of 2 pi / L
    pa = (a.ravel() * (big_l // n0)).astype(np.int64)
    pb = (b.ravel() * (big_l // n1)).astype(np.int64)
    pc = (c.ravel() * (big_l // n2)).astype(np.int64)
    xv = x.ravel()
    n = xv.size
    k0, k1, k2 = (v.ravel().astype(np.int64) for v in np.meshgrid(
        np.arange(n0), np.arange(n1), np.arange(n2), indexing="ij"))
    out = np.empty(n, dtype=np.complex128)
    rows = max(1, chunk_elems // max(n, 1))
    for s in range(0, n, rows):
        e = (k0[s:s + rows, None] * pa[None, :]
             + k1[s:s + rows, None] * pb[None, :]
             + k2[s:s + rows, None] * pc[None, :]) % big_l
        out[s:s + rows] = table[e] @ xv
    return out.reshape(n0, n1, n2)


def brute_dft3_at(x, ks, sign: int = -1) -> np.ndarray:
    """The same sum evaluated only at the listed output indices ks (k, 3)."""
    x = np.asarray(x, dtype=np.complex128)
    n0, n1, n2 = x.shape
    big_l = _lcm(_lcm(n0, n1), n2)
    table = np.exp(sign * 2j * np.pi * np.arange(big_l, dtype=np.float64) / big_l)
    a, b, c = np.meshgrid(np.arange(n0), np.arange(n1), np.arange(n2), indexing="ij")
    pa = (a.ravel() * (big_l // n0)).astype(np.int64)
    pb = (b.ravel() * (big_l // n1)).astype(np.int64)
    pc = (c.ravel() * (big_l // n2)).astype(np.int64)
    xv = x.ravel()
    ks = np.asarray(ks, dtype=np.int64).reshape(-1, 3)
    out = np.empty(len(ks), dtype=np.complex128)
    for i, (q0, q1, q2) in enumerate(ks):
        e = (q0 * pa + q1 * pb + q2 * pc) % big_l
        out[i] = np.dot(table[e], xv)
    return out


def dftnd_at(x, ks, sign: int = -1, chunk_rows: int = 1 << 18) -> np.ndarray:
    """The N-D DFT sum X[k] = sum_a x[a] exp(sign 2 pi i sum_j k_j a_j / n_j)
    evaluated only at the listed outputs ks (S, rank), for arrays too large
    for a full transform.  The exponential of the sum is the product of the
    per-axis exponentials, so the sum is contracted one axis at a time (the
    last axis for all S outputs at once, over row chunks of the leading
    axes, in FP64), against phase vectors whose phases are reduced exactly in
    integers: exp(sign 2 pi i ((k_j a_j) mod n_j) / n_j)."""
    x = np.asarray(x)
    shape = x.shape
    r = x.ndim
    ks = np.asarray(ks, dtype=np.int64).reshape(-1, r)
    n_out = len(ks)

    def phase(j, kcol):
        n = shape[j]
        e = (np.arange(n, dtype=np.int64)[:, None] * np.asarray(kcol, dtype=np.int64)[None, :]) % n
        return np.exp(sign * 2j * np.pi * e / n)

    lead = int(np.prod(shape[:-1], dtype=np.int64))
    flat = x.reshape(lead, shape[-1])
    w_last = phase(r - 1, ks[:, r - 1])
    part = np.empty((lead, n_out), dtype=np.complex128)
    for s in range(0, lead, chunk_rows):
        part[s:s + chunk_rows] = flat[s:s + chunk_rows].astype(np.complex128) @ w_last
    out = np.empty(n_out, dtype=np.complex128)
    for i in range(n_out):
        v = part[:, i].reshape(shape[:-1])
        for j in range(r - 2, -1, -1):
            v = v @ phase(j, [ks[i, j]])[:, 0]
        out[i] = v
    return out
