// registry.hpp -- table of compiled kernel variants, per precision.
#pragma once

#include "kernels.hpp"

namespace mifft {

template <typename T> using ContigFn = void (*)(ContigArgs<T>);
template <typename T> using StridedFn = void (*)(StridedArgs<T>);
template <typename T> using RealFn = void (*)(RealArgs<T>);
template <typename T> using PoissonXFn = void (*)(PoissonXArgs<T>);

// One compiled configuration of a line length: its radix policy, the
// elements-per-thread multiplier and the kernels built from it.
template <typename T> struct Variant {
    int L;
    int policy;
    int emul;
    int tpl;     // threads per line
    int prefetch; // the strided kernel prefetches the next column tile
    int poisson_B; // columns per tile of the fused spectral x-pass (compiled in)
    int nstages;
    int radix[24];
    ContigFn<T> contig;
    ContigFn<T> contig_pack;
    StridedFn<T> strided;
    StridedFn<T> strided_split;  // loads through the unpack map
    StridedFn<T> strided_osplit; // stores through the slab pack map
    RealFn<T> r2c; // line of 2L reals
    RealFn<T> c2r;
    PoissonXFn<T> poisson_x; // fused x-forward, multiply, x-inverse
};

// All variants of this precision (concatenated over the compiled chunks).
template <typename T> const Variant<T>* variant_table(int* count);

} // namespace mifft
