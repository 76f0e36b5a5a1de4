// spectral.hpp -- the multipliers of the spectral operators on the periodic
// box [0, 2 pi)^3 (the "fast spectral operators" of Sec. 1), applied to one
// half-spectrum element.  Shared by the fused x-pass and the standalone
// multiply.  The codes equal the MIFFT_OP_* values of the C ABI.
#pragma once

#include "fft_engine.hpp"

namespace mifft {

enum SpectralOp { OP_POISSON = 0, OP_LAPLACIAN = 1, OP_HELMHOLTZ = 2, OP_DX = 3, OP_DY = 4, OP_DZ = 5 };

// Wavenumber of raw index i on an axis of n points: i below n/2, else i - n.
__device__ __forceinline__ int signed_k(int i, int n) { return 2 * i < n ? i : i - n; }

// What the multiplier needs of a column (fixed i1, i2) of the half spectrum
// of an n0 x n1 x n2 real grid: k1^2 + k2^2, and for d/dy, d/dz the factor
// k_j scale (0 at the Nyquist index i_j = n_j/2 of an even axis).
template <typename T> struct SpectralCol {
    int kk12;
    T c;
};

template <typename T>
__device__ __forceinline__ SpectralCol<T> spectral_col(int op, int i1, int i2, int n1, int n2, T scale)
{
    const int k1 = signed_k(i1, n1), k2 = i2;
    SpectralCol<T> s;
    s.kk12 = k1 * k1 + k2 * k2;
    s.c = T(0);
    if (op == OP_DY && 2 * i1 != n1) s.c = (T)k1 * scale;
    if (op == OP_DZ && 2 * i2 != n2) s.c = (T)k2 * scale;
    return s;
}

// v * m(k) * scale for element i0 (of n0) of a column:
//   Poisson    -1/|k|^2, 0 at k = 0         Laplacian  -|k|^2
//   Helmholtz  1/(alpha + |k|^2), 0 where alpha + |k|^2 = 0
//   d/dx_j     i k_j, 0 at i_j = n_j/2 (the Nyquist mode of an even axis)
template <typename T>
__device__ __forceinline__ cx<T> spectral_mul(int op, int i0, int n0, SpectralCol<T> col, T scale, T alpha,
                                              cx<T> v)
{
    const int k0 = signed_k(i0, n0);
    if (op >= OP_DX) {
        T c = col.c;
        if (op == OP_DX) c = (2 * i0 == n0) ? T(0) : (T)k0 * scale;
        return cx<T>{-c * v.y, c * v.x};
    }
    const int kk = k0 * k0 + col.kk12;
    T f;
    if (op == OP_LAPLACIAN) {
        f = -(T)kk * scale;
    } else if (op == OP_HELMHOLTZ) {
        const T den = alpha + (T)kk;
        f = den == T(0) ? T(0) : scale / den;
    } else {
        f = kk == 0 ? T(0) : -scale / (T)kk;
    }
    return cx<T>{v.x * f, v.y * f};
}

} // namespace mifft
