// aux_kernels.hip -- twiddle generation, spectral Poisson multiply, standalone
// pack / unpack of the row all-to-all, and a plain copy.
#include "aux_kernels.hpp"
#include "spectral.hpp"

namespace mifft {

// w[m] = exp(-2 pi i m / n), m = 0 .. n-1, evaluated in FP64 and rounded to
// nearest in T.  The angle is split exactly in integers into whole quarter
// turns q and a remainder; the remainder angle is folded into [0, pi/4] so
// sincospi only sees a small argument, and multiples of a quarter turn give
// exact 0 and +-1.
template <typename T> __global__ void k_twiddles(cx<T>* w, int n)
{
    const int m = blockIdx.x * blockDim.x + threadIdx.x;
    if (m >= n) return;
    const long long q = (4LL * m) / n;
    const long long r = 4LL * m - q * n;
    double s, c;
    if (2 * r <= n) {
        sincospi((double)r / (2.0 * (double)n), &s, &c);
    } else {
        double s2, c2;
        sincospi((double)(n - r) / (2.0 * (double)n), &s2, &c2);
        s = c2;
        c = s2;
    }
    double cr, sr; // cos, sin of the full angle 2 pi m / n
    switch ((int)q) {
    case 0: cr = c; sr = s; break;
    case 1: cr = -s; sr = c; break;
    case 2: cr = -c; sr = -s; break;
    default: cr = s; sr = -c; break;
    }
    w[m] = cx<T>{(T)cr, (T)(-sr)};
}

template <typename T>
hipError_t launch_twiddles(cx<T>* w, int n, hipStream_t s)
{
    if (n <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_twiddles<T>, dim3((n + 255) / 256), dim3(256), 0, s, w, n);
    return hipGetLastError();
}

// Standalone spectral multiply on the half spectrum [n0][n1][n2c] of an
// n0 x n1 x n2 real grid: dst = m(k) src (dst += m(k) src with acc), m from
// spectral_mul; src may equal dst.
template <typename T>
__global__ void k_spectral(const cx<T>* src, cx<T>* dst, int n0, int n1, int n2c, int n2, int op, T scale,
                           T alpha, int acc, long long total)
{
    const long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= total) return;
    const int i2 = (int)(i % n2c);
    const long long r = i / n2c;
    const int i1 = (int)(r % n1);
    const int i0 = (int)(r / n1);
    cx<T> v = spectral_mul<T>(op, i0, n0, spectral_col<T>(op, i1, i2, n1, n2, scale), scale, alpha, src[i]);
    if (acc) {
        const cx<T> o = dst[i];
        v.x += o.x;
        v.y += o.y;
    }
    dst[i] = v;
}

template <typename T>
hipError_t launch_spectral(const cx<T>* src, cx<T>* dst, int n0, int n1, int n2c, int n2, int op, T scale,
                           T alpha, int acc, hipStream_t s)
{
    const long long total = (long long)n0 * n1 * n2c;
    if (total == 0) return hipSuccess;
    hipLaunchKernelGGL(k_spectral<T>, dim3((unsigned)((total + 255) / 256)), dim3(256), 0, s, src, dst, n0,
                       n1, n2c, n2, op, scale, alpha, acc, total);
    return hipGetLastError();
}

// Pack: S[j][i0][i1][m] = A[i0][i1][j*M + m].  One thread per element of S;
// a run of M contiguous elements of A becomes a run of M in S.
template <typename T>
__global__ void k_pack(const cx<T>* __restrict__ a, cx<T>* __restrict__ s, long long lines, int p1,
                       int M, long long total)
{
    const long long o = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (o >= total) return;
    const int m = (int)(o % M);
    const long long rest = o / M;
    const long long line = rest % lines; // i0 * n1l + i1
    const int j = (int)(rest / lines);
    s[o] = a[line * ((long long)p1 * M) + (long long)j * M + m];
}

// Unpack: B[i0][j*n1l + i1][m] = R[j][i0][i1][m].  One thread per element of B.
template <typename T>
__global__ void k_unpack(const cx<T>* __restrict__ r, cx<T>* __restrict__ b, int n0l, int n1l,
                         int p1, int M, long long total)
{
    const long long o = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (o >= total) return;
    const int m = (int)(o % M);
    const long long rest = o / M;
    const int y = (int)(rest % ((long long)p1 * n1l));
    const int i0 = (int)(rest / ((long long)p1 * n1l));
    const int j = y / n1l;
    const int i1 = y - j * n1l;
    b[o] = r[(((long long)j * n0l + i0) * n1l + i1) * M + m];
}

template <typename T>
hipError_t launch_pack(const cx<T>* a, cx<T>* s, int n0l, int n1l, int p1, int M, hipStream_t st)
{
    const long long lines = (long long)n0l * n1l;
    const long long total = lines * p1 * M;
    if (total == 0) return hipSuccess;
    hipLaunchKernelGGL(k_pack<T>, dim3((unsigned)((total + 255) / 256)), dim3(256), 0, st, a, s,
                       lines, p1, M, total);
    return hipGetLastError();
}

template <typename T>
hipError_t launch_unpack(const cx<T>* r, cx<T>* b, int n0l, int n1l, int p1, int M, hipStream_t st)
{
    const long long total = (long long)n0l * n1l * p1 * M;
    if (total == 0) return hipSuccess;
    hipLaunchKernelGGL(k_unpack<T>, dim3((unsigned)((total + 255) / 256)), dim3(256), 0, st, r, b,
                       n0l, n1l, p1, M, total);
    return hipGetLastError();
}

__global__ void k_copy16(const uint4* __restrict__ a, uint4* __restrict__ b, long long n16)
{
    for (long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x; i < n16;
         i += (long long)gridDim.x * blockDim.x)
        b[i] = a[i];
}

__global__ void k_copy1(const unsigned char* __restrict__ a, unsigned char* __restrict__ b, long long n)
{
    const long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) b[i] = a[i];
}

hipError_t launch_copy(const void* src, void* dst, size_t bytes, hipStream_t s)
{
    if (bytes == 0 || src == dst) return hipSuccess;
    const bool vec = ((uintptr_t)src % 16 == 0) && ((uintptr_t)dst % 16 == 0) && (bytes % 16 == 0);
    if (vec) {
        const long long n16 = (long long)(bytes / 16);
        long long blocks = (n16 + 255) / 256;
        if (blocks > 65536) blocks = 65536;
        hipLaunchKernelGGL(k_copy16, dim3((unsigned)blocks), dim3(256), 0, s, (const uint4*)src,
                           (uint4*)dst, n16);
    } else {
        hipLaunchKernelGGL(k_copy1, dim3((unsigned)((bytes + 255) / 256)), dim3(256), 0, s,
                           (const unsigned char*)src, (unsigned char*)dst, (long long)bytes);
    }
    return hipGetLastError();
}

// Tile copy with a strided pass's access pattern and no arithmetic: tile
// (group g, columns c0 .. c0 + B - 1) of L rows; thread (t, c) moves rows t,
// t + T, ... of column c0 + c, 16 loads in flight before their stores.  The
// copy rate it reaches is the ceiling of that access pattern on the device
// (a reference for the strided FFT passes' roofline fraction).  NTL / NTS:
// streaming (non-temporal) loads / stores, as the FFT passes use them.
template <typename T, bool NTL, bool NTS>
__global__ __launch_bounds__(1024) void k_tile_copy(const cx<T>* __restrict__ in, cx<T>* __restrict__ out, int L,
                                                  int cols, int groups, int B, int TT, int tpg, long long es_in,
                                                  long long es_out, long long gs_in, long long gs_out)
{
    typedef typename nt_vec2<T>::type N2;
    const int g = (int)blockIdx.x / tpg;
    const int col = ((int)blockIdx.x - g * tpg) * B + (int)threadIdx.x % B;
    const int t = (int)threadIdx.x / B;
    if (g >= groups || col >= cols) return;
    const cx<T>* src = in + (long long)g * gs_in + col;
    cx<T>* dst = out + (long long)g * gs_out + col;
    constexpr int K = 16;
    for (int base = t; base < L; base += K * TT) {
        N2 v[K];
#pragma unroll
        for (int k = 0; k < K; ++k) {
            const int r = base + k * TT;
            if (r < L) {
                const N2* q = reinterpret_cast<const N2*>(src + (long long)r * es_in);
                if constexpr (NTL)
                    v[k] = __builtin_nontemporal_load(q);
                else
                    v[k] = *q;
            }
        }
#pragma unroll
        for (int k = 0; k < K; ++k) {
            const int r = base + k * TT;
            if (r < L) {
                N2* q = reinterpret_cast<N2*>(dst + (long long)r * es_out);
                if constexpr (NTS)
                    __builtin_nontemporal_store(v[k], q);
                else
                    *q = v[k];
            }
        }
    }
}

template <typename T>
hipError_t launch_tile_copy(const cx<T>* in, cx<T>* out, int L, int cols, int groups, int B, int TT, long long es_in,
                            long long es_out, long long gs_in, long long gs_out, unsigned flags, hipStream_t s)
{
    const int tpg = (cols + B - 1) / B;
    const long long tiles = (long long)tpg * groups;
    if (tiles == 0) return hipSuccess;
    auto fn = (flags & 3u) == 3u ? k_tile_copy<T, true, true>
              : (flags & 1u)     ? k_tile_copy<T, true, false>
              : (flags & 2u)     ? k_tile_copy<T, false, true>
                                 : k_tile_copy<T, false, false>;
    hipLaunchKernelGGL(fn, dim3((unsigned)tiles), dim3(B * TT), 0, s, in, out, L, cols, groups, B, TT, tpg, es_in,
                       es_out, gs_in, gs_out);
    return hipGetLastError();
}

// Contiguous reference copy of n16 16-byte words: each thread moves U words
// per grid-stride round (all loads issued before the stores), with optional
// streaming loads / stores -- the best plain copy this device reaches, the
// achievable ceiling the passes' bandwidth is read against.
template <bool NTL, bool NTS>
__global__ __launch_bounds__(256) void k_copy_ref(const uint4* __restrict__ a, uint4* __restrict__ b, long long n16)
{
    typedef unsigned int U4 __attribute__((ext_vector_type(4)));
    constexpr int U = 4;
    const long long stride = (long long)gridDim.x * blockDim.x;
    for (long long i0 = (long long)blockIdx.x * blockDim.x + threadIdx.x; i0 < n16; i0 += U * stride) {
        U4 v[U];
#pragma unroll
        for (int u = 0; u < U; ++u) {
            const long long i = i0 + u * stride;
            if (i < n16) {
                const U4* q = reinterpret_cast<const U4*>(a + i);
                if constexpr (NTL)
                    v[u] = __builtin_nontemporal_load(q);
                else
                    v[u] = *q;
            }
        }
#pragma unroll
        for (int u = 0; u < U; ++u) {
            const long long i = i0 + u * stride;
            if (i < n16) {
                U4* q = reinterpret_cast<U4*>(b + i);
                if constexpr (NTS)
                    __builtin_nontemporal_store(v[u], q);
                else
                    *q = v[u];
            }
        }
    }
}

// Blocked reference copy: workgroup b copies the contiguous block of
// 4 x 128 words at b x 512 (8 KiB, as one z-pass workgroup of two 512-point
// complex64 lines reads and then writes), all four loads of a thread before
// its stores.  The last block may be partial.
template <bool NTL, bool NTS>
__global__ __launch_bounds__(128) void k_copy_blk(const uint4* __restrict__ a, uint4* __restrict__ b, long long n16)
{
    typedef unsigned int U4 __attribute__((ext_vector_type(4)));
    constexpr int U = 4;
    const long long base = (long long)blockIdx.x * (U * 128) + threadIdx.x;
    U4 v[U];
#pragma unroll
    for (int u = 0; u < U; ++u) {
        const long long i = base + u * 128;
        if (i < n16) {
            const U4* q = reinterpret_cast<const U4*>(a + i);
            if constexpr (NTL)
                v[u] = __builtin_nontemporal_load(q);
            else
                v[u] = *q;
        }
    }
#pragma unroll
    for (int u = 0; u < U; ++u) {
        const long long i = base + u * 128;
        if (i < n16) {
            U4* q = reinterpret_cast<U4*>(b + i);
            if constexpr (NTS)
                __builtin_nontemporal_store(v[u], q);
            else
                *q = v[u];
        }
    }
}

hipError_t launch_copy_ref(const void* src, void* dst, size_t bytes, unsigned flags, int grid, hipStream_t s)
{
    const long long n16 = (long long)(bytes / 16);
    if (n16 == 0) return hipSuccess;
    if (flags & 4u) { // blocked: one 8 KiB block per workgroup (grid ignored)
        const long long blocks = (n16 + 511) / 512;
        auto fb = (flags & 3u) == 3u ? k_copy_blk<true, true>
                  : (flags & 1u)     ? k_copy_blk<true, false>
                  : (flags & 2u)     ? k_copy_blk<false, true>
                                     : k_copy_blk<false, false>;
        if (blocks > 0x7fffffffLL) return hipErrorInvalidValue;
        hipLaunchKernelGGL(fb, dim3((unsigned)blocks), dim3(128), 0, s, (const uint4*)src, (uint4*)dst, n16);
        return hipGetLastError();
    }
    long long blocks = grid > 0 ? grid : (n16 + 4 * 256 - 1) / (4 * 256);
    if (blocks > (1LL << 30)) blocks = 1LL << 30;
    auto fn = (flags & 3u) == 3u ? k_copy_ref<true, true>
              : (flags & 1u)     ? k_copy_ref<true, false>
              : (flags & 2u)     ? k_copy_ref<false, true>
                                 : k_copy_ref<false, false>;
    hipLaunchKernelGGL(fn, dim3((unsigned)blocks), dim3(256), 0, s, (const uint4*)src, (uint4*)dst, n16);
    return hipGetLastError();
}

template hipError_t launch_tile_copy<float>(const cx<float>*, cx<float>*, int, int, int, int, int, long long,
                                            long long, long long, long long, unsigned, hipStream_t);
template hipError_t launch_tile_copy<double>(const cx<double>*, cx<double>*, int, int, int, int, int, long long,
                                             long long, long long, long long, unsigned, hipStream_t);
template hipError_t launch_twiddles<float>(cx<float>*, int, hipStream_t);
template hipError_t launch_twiddles<double>(cx<double>*, int, hipStream_t);
template hipError_t launch_spectral<float>(const cx<float>*, cx<float>*, int, int, int, int, int, float, float,
                                           int, hipStream_t);
template hipError_t launch_spectral<double>(const cx<double>*, cx<double>*, int, int, int, int, int, double,
                                            double, int, hipStream_t);
template hipError_t launch_pack<float>(const cx<float>*, cx<float>*, int, int, int, int, hipStream_t);
template hipError_t launch_pack<double>(const cx<double>*, cx<double>*, int, int, int, int, hipStream_t);
template hipError_t launch_unpack<float>(const cx<float>*, cx<float>*, int, int, int, int, hipStream_t);
template hipError_t launch_unpack<double>(const cx<double>*, cx<double>*, int, int, int, int,
                                          hipStream_t);

} // namespace mifft
