// aux_kernels.hpp -- host launchers of the auxiliary kernels.
#pragma once

#include "fft_engine.hpp"

namespace mifft {

template <typename T> hipError_t launch_twiddles(cx<T>* w, int n, hipStream_t s);
template <typename T>
hipError_t launch_spectral(const cx<T>* src, cx<T>* dst, int n0, int n1, int n2c, int n2, int op, T scale,
                           T alpha, int acc, hipStream_t s);
template <typename T>
hipError_t launch_pack(const cx<T>* a, cx<T>* s, int n0l, int n1l, int p1, int M, hipStream_t st);
template <typename T>
hipError_t launch_unpack(const cx<T>* r, cx<T>* b, int n0l, int n1l, int p1, int M, hipStream_t st);
hipError_t launch_copy(const void* src, void* dst, size_t bytes, hipStream_t s);
template <typename T>
hipError_t launch_tile_copy(const cx<T>* in, cx<T>* out, int L, int cols, int groups, int B, int TT, long long es_in,
                            long long es_out, long long gs_in, long long gs_out, unsigned flags, hipStream_t s);
hipError_t launch_copy_ref(const void* src, void* dst, size_t bytes, unsigned flags, int grid, hipStream_t s);

// 2-vectors of T for the streaming-load / -store builtins
template <typename T> struct nt_vec2;
template <> struct nt_vec2<float> { typedef float type __attribute__((ext_vector_type(2))); };
template <> struct nt_vec2<double> { typedef double type __attribute__((ext_vector_type(2))); };

} // namespace mifft
