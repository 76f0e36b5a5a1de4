"""FP64 CPU oracle for the local phases of the pencil 3-D FFT (AccFFT, Sec. 2).

TEST INFRASTRUCTURE ONLY.  Only the test suite, the smoke check and the CPU
baseline leg of the benchmark may import this package.  The product path (the
HIP library and its Python binding) never imports, loads or calls it, and it
shares no code with that path.

Contents
  * ``fft3d_c2c / fft3d_r2c / fft3d_c2r / fft_axis`` -- ctypes wrappers around
    ``oracle_fft.c`` (row-column mixed-radix Cooley-Tukey, Algorithm 1 order).
  * ``poisson_half / poisson_solve`` -- the spectral Poisson operator
    (Sec. 1 lists "fast spectral operators"; the operator is the textbook
    periodic solve -1/|k|^2 with the k = 0 mode zeroed).
  * ``pencil_pack / pencil_unpack / pencil_share_forward`` -- the pack, loopback
    exchange and unpack maps of the row all-to-all (Sec. 2, pencil paragraph,
    and Algorithm 1 up to the y-FFT), written as numpy permutations.
  * ``slab_pack / slab_forward / slab_inverse`` -- the slab decomposition of
    Algorithm 3 for all tasks at once, the all-to-all done as array copies;
    ``c2r_z`` is the z-only C2R its inverse ends with.
  * ``fftnd_c2c / fftnd_r2c / fftnd_c2r`` -- transforms of any rank in the
    axis order of Algorithm 2 (last axis first; the inverse first axis first).
  * ``spectral_multiplier / spectral_apply / gradient / divergence`` -- more
    of the "fast spectral operators" of Sec. 1 on the periodic box: Laplacian,
    Helmholtz solve, partial derivatives (the even-length Nyquist mode of a
    derivative set to zero), gradient and divergence.
  * ``brute`` submodule -- the direct O(N^2) DFT used to pin the FFT.

Conventions (readings of the paper, listed in the design notes): forward uses
exp(-2 pi i ...), inverse exp(+2 pi i ...), neither is scaled; arrays are
C-order [x][y][z] in both domains; R2C keeps k2 = 0 .. n2 // 2.

Parity status: every function here is pinned by the CPU tests; none is
parity unpinned.
"""
from __future__ import annotations

import ctypes
import os
import subprocess
import threading

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "oracle_fft.c")
_LIB = os.path.join(_HERE, "liboracle_fft.so")
_lock = threading.Lock()
_lib = None


def build(force: bool = True) -> str:
    """Compile ``oracle_fft.c`` into ``liboracle_fft.so`` with gcc + OpenMP."""
    if not force and os.path.exists(_LIB) and os.path.getmtime(_LIB) >= os.path.getmtime(_SRC):
        return _LIB
    tmp = _LIB + ".tmp%d" % os.getpid()
    cmd = ["gcc", "-O2", "-fopenmp", "-fPIC", "-shared", "-std=c11", "-Wall",
           "-o", tmp, _SRC, "-lm"]
    subprocess.run(cmd, check=True)
    os.replace(tmp, _LIB)
    return _LIB


def _load():
    global _lib
    with _lock:
        if _lib is None:
            if not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
                build(force=True)
            lib = ctypes.CDLL(_LIB)
            dp = ctypes.POINTER(ctypes.c_double)
            i64 = ctypes.c_int64
            ci = ctypes.c_int
            lib.oracle_fft3d_c2c.argtypes = [dp, ci, ci, ci, ci]
            lib.oracle_fft_axis.argtypes = [dp, i64, ci, i64, ci]
            lib.oracle_fft3d_r2c.argtypes = [dp, dp, ci, ci, ci]
            lib.oracle_fft3d_c2r.argtypes = [dp, dp, ci, ci, ci]
            lib.oracle_c2r_z.argtypes = [dp, dp, i64, ci]
            lib.oracle_poisson_half.argtypes = [dp, ci, ci, ci, ctypes.c_double]
            lib.oracle_max_threads.argtypes = []
            lib.oracle_max_threads.restype = ci
            for f in (lib.oracle_fft3d_c2c, lib.oracle_fft_axis,
                      lib.oracle_fft3d_r2c, lib.oracle_fft3d_c2r, lib.oracle_c2r_z,
                      lib.oracle_poisson_half):
                f.restype = None
            _lib = lib
    return _lib


def max_threads() -> int:
    """Threads the oracle's OpenMP loops use on this host."""
    return int(_load().oracle_max_threads())


def _dptr(a: np.ndarray):
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_double))


def _as_c128(x) -> np.ndarray:
    return np.ascontiguousarray(np.asarray(x), dtype=np.complex128).copy()


def fft3d_c2c(x, sign: int = -1) -> np.ndarray:
    """Unscaled 3-D DFT, z then y then x (Algorithm 1, left column)."""
    a = _as_c128(x)
    n0, n1, n2 = a.shape
    _load().oracle_fft3d_c2c(_dptr(a), n0, n1, n2, int(sign))
    return a


def fft_axis(x, axis: int, sign: int = -1) -> np.ndarray:
    """Unscaled 1-D DFT along one axis of an N-D complex array."""
    a = _as_c128(x)
    shape = a.shape
    outer = int(np.prod(shape[:axis], dtype=np.int64))
    inner = int(np.prod(shape[axis + 1:], dtype=np.int64))
    _load().oracle_fft_axis(_dptr(a), outer, shape[axis], inner, int(sign))
    return a


def fft3d_r2c(x) -> np.ndarray:
    """Real [n0][n1][n2] -> half spectrum [n0][n1][n2//2+1], unscaled."""
    a = np.ascontiguousarray(np.asarray(x), dtype=np.float64)
    n0, n1, n2 = a.shape
    out = np.empty((n0, n1, n2 // 2 + 1), dtype=np.complex128)
    _load().oracle_fft3d_r2c(_dptr(a), _dptr(out), n0, n1, n2)
    return out


def fft3d_c2r(y, n2: int) -> np.ndarray:
    """Half spectrum [n0][n1][n2//2+1] -> real [n0][n1][n2], unscaled; the
    imaginary parts at k2 = 0 and (even n2) k2 = n2/2 are discarded."""
    a = _as_c128(y)
    n0, n1, n2c = a.shape
    if n2c != n2 // 2 + 1:
        raise ValueError("half spectrum has %d entries along z, n2=%d needs %d"
                         % (n2c, n2, n2 // 2 + 1))
    out = np.empty((n0, n1, n2), dtype=np.float64)
    _load().oracle_fft3d_c2r(_dptr(a), _dptr(out), n0, n1, n2)
    return out


def c2r_z(y, n2: int) -> np.ndarray:
    """z-only C2R: half lines [..., n2//2+1] -> real lines [..., n2], unscaled,
    by the C2R definition (imaginary parts at k2 = 0 and, for even n2,
    k2 = n2/2 discarded); the x and y axes are left alone."""
    a = _as_c128(y)
    n2c = a.shape[-1]
    if n2c != n2 // 2 + 1:
        raise ValueError("half lines have %d entries, n2=%d needs %d" % (n2c, n2, n2 // 2 + 1))
    lines = int(np.prod(a.shape[:-1], dtype=np.int64))
    out = np.empty(a.shape[:-1] + (n2,), dtype=np.float64)
    _load().oracle_c2r_z(_dptr(a), _dptr(out), lines, n2)
    return out


def poisson_half(yhat, n2: int, scale: float = 1.0) -> np.ndarray:
    """U = -scale * F / |k|^2 on the half spectrum, U[0,0,0] = 0."""
    a = _as_c128(yhat)
    n0, n1, n2c = a.shape
    if n2c != n2 // 2 + 1:
        raise ValueError("bad half-spectrum shape")
    _load().oracle_poisson_half(_dptr(a), n0, n1, n2, float(scale))
    return a


def poisson_solve(f) -> np.ndarray:
    """Periodic Poisson solve lap(u) = f on [0, 2 pi)^3: R2C, multiply by
    -1/|k|^2 (k = 0 zeroed), C2R, divide by N."""
    f = np.asarray(f, dtype=np.float64)
    n0, n1, n2 = f.shape
    n = n0 * n1 * n2
    fh = fft3d_r2c(f)
    uh = poisson_half(fh, n2, 1.0)
    return fft3d_c2r(uh, n2) / n


# ---- pencil share: pack, loopback exchange, unpack (Algorithm 1, up to the y-FFT) ----

def pencil_pack(ahat, p1: int) -> np.ndarray:
    """Row all-to-all send layout S[j][i0][i1][m] = Ahat[i0][i1][j*M + m] with
    M = n2 / p1: block j holds the k2 range destined for row peer j."""
    a = np.asarray(ahat)
    n0l, n1l, n2 = a.shape
    if n2 % p1:
        raise ValueError("p1 must divide n2")
    m = n2 // p1
    return np.ascontiguousarray(a.reshape(n0l, n1l, p1, m).transpose(2, 0, 1, 3))


def pencil_unpack(r, n1l: int) -> np.ndarray:
    """Receive layout R[j][i0][i1][m] -> B[i0][j*n1l + i1][m]: the block from
    row peer j supplies the y range j*n1l .. (j+1)*n1l."""
    r = np.asarray(r)
    p1, n0l, n1l_, m = r.shape
    if n1l_ != n1l:
        raise ValueError("receive block has the wrong y extent")
    return np.ascontiguousarray(r.transpose(1, 0, 2, 3).reshape(n0l, p1 * n1l, m))


def pencil_share_forward(a, p1: int) -> np.ndarray:
    """One rank's local phases with a loopback exchange: z-DFT of the
    n0l x n1l x n2 share, pack, receive buffer = send buffer, unpack, then the
    y-DFT of length p1 * n1l along axis 1."""
    a = np.asarray(a)
    n0l, n1l, n2 = a.shape
    ahat = fft_axis(a, 2, -1)
    s = pencil_pack(ahat, p1)
    b = pencil_unpack(s, n1l)
    return fft_axis(b, 1, -1)


# ---- slab decomposition (Algorithm 3): P tasks, each holding N0/P x-planes ----

def slab_pack(ahat, p: int) -> np.ndarray:
    """Send layout of the forward slab transpose: S[j][i0][i1][k2] =
    Ahat[i0][j*n1l + i1][k2] with n1l = N1/p, so block j holds the y range
    that task j owns after the exchange (the transpose of Algorithm 3)."""
    a = np.asarray(ahat)
    n0l, n1, nc = a.shape
    if n1 % p:
        raise ValueError("p must divide N1")
    return np.ascontiguousarray(a.reshape(n0l, p, n1 // p, nc).transpose(1, 0, 2, 3))


def slab_forward(x, p: int, real: bool = False) -> list:
    """Algorithm 3, forward, for all p tasks with the all-to-all done as
    array copies.  Task r holds the slab x[r*N0/p : (r+1)*N0/p]; it computes
    the 2-D DFTs of its x-planes (z, R2C if `real`, then y), sends block j of
    its pack to task j, stacks the received blocks in sender order along x
    (N0 x N1/p x N2c) and finishes with the x-DFT.  Returns the p spectral
    shares; share j is X[:, j*N1/p : (j+1)*N1/p, :]."""
    x = np.asarray(x)
    n0, n1, n2 = x.shape
    if n0 % p or n1 % p:
        raise ValueError("p must divide N0 and N1")
    n0l = n0 // p
    sends = []
    for r in range(p):
        a = x[r * n0l:(r + 1) * n0l]
        if real:
            ahat = fft_axis(np.asarray(a, dtype=np.float64), 2, -1)[..., :n2 // 2 + 1]
        else:
            ahat = fft_axis(a, 2, -1)
        ahat = fft_axis(ahat, 1, -1)
        sends.append(slab_pack(ahat, p))
    shares = []
    for j in range(p):
        b = np.concatenate([sends[s][j] for s in range(p)], axis=0)
        shares.append(fft_axis(b, 0, -1))
    return shares


def slab_inverse(shares, p: int, n2: int = None) -> list:
    """Algorithm 3, inverse: each task's N0 x N1/p x N2c share gets the x-IDFT;
    block r of it (x rows r*N0/p ...) goes to task r, which places the block
    from task s at y rows s*N1/p ... (the receive map of the pencil unpack),
    then runs the y-IDFT and the z-IDFT (the z-only C2R when n2 is given).
    Unscaled.  Returns the p spatial slabs."""
    if len(shares) != p:
        raise ValueError("need one share per task")
    n0 = np.asarray(shares[0]).shape[0]
    if n0 % p:
        raise ValueError("p must divide N0")
    n0l = n0 // p
    sent = [fft_axis(s, 0, +1) for s in shares]
    slabs = []
    for r in range(p):
        recv = np.stack([sent[s][r * n0l:(r + 1) * n0l] for s in range(p)])
        a = pencil_unpack(recv, recv.shape[2])
        a = fft_axis(a, 1, +1)
        slabs.append(c2r_z(a, n2) if n2 is not None else fft_axis(a, 2, +1))
    return slabs


# ---- arrays of any rank (Algorithm 2 with every P_i = 1) ----

def fftnd_c2c(x, sign: int = -1) -> np.ndarray:
    """Unscaled N-D DFT: 1-D DFTs along the last axis, then along each earlier
    axis in turn (the forward loop of Algorithm 2); the inverse (sign = +1)
    runs the axes first to last, as Algorithm 2's inverse does."""
    a = _as_c128(x)
    order = range(a.ndim - 1, -1, -1) if sign < 0 else range(a.ndim)
    for ax in order:
        a = fft_axis(a, ax, sign)
    return a


def fftnd_r2c(x) -> np.ndarray:
    """Real N-D array -> half spectrum (last axis n//2 + 1), unscaled."""
    a = np.asarray(x, dtype=np.float64)
    n = a.shape[-1]
    a = fft_axis(a, a.ndim - 1, -1)[..., :n // 2 + 1]
    for ax in range(a.ndim - 2, -1, -1):
        a = fft_axis(a, ax, -1)
    return a


def fftnd_c2r(y, n_last: int) -> np.ndarray:
    """Half spectrum -> real N-D array, unscaled: inverse DFTs along the first
    axes in order, then the C2R of the last axis (imaginary parts at k = 0
    and n/2 discarded)."""
    a = _as_c128(y)
    for ax in range(a.ndim - 1):
        a = fft_axis(a, ax, +1)
    return c2r_z(a, n_last)


# ---- spectral operators on [0, 2 pi)^3 (Sec. 1, "fast spectral operators") ----

OP_POISSON, OP_LAPLACIAN, OP_HELMHOLTZ, OP_DX, OP_DY, OP_DZ = 0, 1, 2, 3, 4, 5


def spectral_multiplier(shape, op: int, alpha: float = 0.0) -> np.ndarray:
    """The multiplier m(k) on the half spectrum [n0][n1][n2//2+1] of a real
    [n0][n1][n2] grid.  Integer wavenumbers: k0 = i0 for i0 < n0/2, else
    i0 - n0 (likewise k1); k2 = i2 >= 0.
      OP_POISSON    -1/|k|^2 (0 at k = 0): u solves lap(u) = f
      OP_LAPLACIAN  -|k|^2: u = lap(f)
      OP_HELMHOLTZ  1/(alpha + |k|^2) (0 where that vanishes): u solves
                    alpha u - lap(u) = f
      OP_DX/DY/DZ   i k_j: u = d f / d x_j; for an even n_j the mode
                    i_j = n_j/2 is set to 0 (its sign is ambiguous and the
                    derivative of a real field must stay real)."""
    n0, n1, n2 = shape
    i0 = np.arange(n0)[:, None, None]
    i1 = np.arange(n1)[None, :, None]
    i2 = np.arange(n2 // 2 + 1)[None, None, :]
    k0 = np.where(2 * i0 < n0, i0, i0 - n0).astype(np.float64)
    k1 = np.where(2 * i1 < n1, i1, i1 - n1).astype(np.float64)
    k2 = i2.astype(np.float64)
    kk = k0 ** 2 + k1 ** 2 + k2 ** 2
    full = (n0, n1, n2 // 2 + 1)
    if op == OP_POISSON:
        with np.errstate(divide="ignore"):
            m = np.where(kk == 0, 0.0, -1.0 / np.where(kk == 0, 1.0, kk))
    elif op == OP_LAPLACIAN:
        m = -kk
    elif op == OP_HELMHOLTZ:
        den = alpha + kk
        m = np.where(den == 0, 0.0, 1.0 / np.where(den == 0, 1.0, den))
    elif op in (OP_DX, OP_DY, OP_DZ):
        j = op - OP_DX
        k, i, n = ((k0, i0, n0), (k1, i1, n1), (k2, i2, n2))[j]
        m = np.where(2 * i == n, 0.0, 1j * k)
    else:
        raise ValueError("unknown operator %d" % op)
    return np.broadcast_to(m, full).astype(np.complex128)


def spectral_apply(f, op: int, alpha: float = 0.0) -> np.ndarray:
    """u = C2R(m * R2C(f)) / N: the operator applied to a real periodic field."""
    f = np.asarray(f, dtype=np.float64)
    n = f.size
    return fft3d_c2r(fft3d_r2c(f) * spectral_multiplier(f.shape, op, alpha), f.shape[2]) / n


def gradient(f) -> list:
    """(df/dx0, df/dx1, df/dx2) of a real periodic field."""
    return [spectral_apply(f, op) for op in (OP_DX, OP_DY, OP_DZ)]


def divergence(v0, v1, v2) -> np.ndarray:
    """d v0/dx0 + d v1/dx1 + d v2/dx2, summed in the spectrum and brought back
    with one C2R."""
    v = [np.asarray(a, dtype=np.float64) for a in (v0, v1, v2)]
    shape = v[0].shape
    acc = sum(fft3d_r2c(a) * spectral_multiplier(shape, op)
              for a, op in zip(v, (OP_DX, OP_DY, OP_DZ)))
    return fft3d_c2r(acc, shape[2]) / v[0].size
