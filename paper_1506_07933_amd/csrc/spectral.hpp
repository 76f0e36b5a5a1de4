// spectral.hpp -- the multipliers of the spectral operators on the periodic
// box [0, 2 pi)^3 (the "fast spectral operators" of Sec. 1), applied to one
// half-spectrum element.  Shared by the fused x-pass and the standalone
// multiply.  The codes equal the MIFFT_OP_* values of the C ABI.
#pragma once

#include "fft_engine.hpp"

namespace mifft {

enum SpectralOp { OP_POISSON = 0, OP_LAPLACIAN = 1, OP_HELMHOLTZ = 2, OP_DX = 3, OP_DY = 4, OP_DZ = 5 };

// v * m(k) * scale for the element at raw indices (i0, i1, i2) of the half
// spectrum of an n0 x n1 x n2 real grid.  Wavenumbers k0 = i0 below n0/2,
// else i0 - n0 (likewise k1); k2 = i2.
//   Poisson    -1/|k|^2, 0 at k = 0         Laplacian  -|k|^2
//   Helmholtz  1/(alpha + |k|^2), 0 where alpha + |k|^2 = 0
//   d/dx_j     i k_j, 0 at i_j = n_j/2 (the Nyquist mode of an even axis)
template <typename T>
__device__ __forceinline__ cx<T> spectral_mul(int op, long long i0, long long i1, long long i2, long long n0,
                                              long long n1, long long n2, T scale, T alpha, cx<T> v)
{
    const long long k0 = (2 * i0 < n0) ? i0 : i0 - n0;
    const long long k1 = (2 * i1 < n1) ? i1 : i1 - n1;
    const long long k2 = i2;
    if (op >= OP_DX) {
        long long k, i, n;
        if (op == OP_DX) {
            k = k0, i = i0, n = n0;
        } else if (op == OP_DY) {
            k = k1, i = i1, n = n1;
        } else {
            k = k2, i = i2, n = n2;
        }
        const T c = (2 * i == n) ? T(0) : (T)k * scale;
        return cx<T>{-c * v.y, c * v.x};
    }
    const long long kk = k0 * k0 + k1 * k1 + k2 * k2;
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
