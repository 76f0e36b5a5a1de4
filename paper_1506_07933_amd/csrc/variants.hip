// variants.hip -- explicit instantiation of the kernels for one chunk of the
// compiled axis lengths.  Built once per (precision, chunk) with
// -DMIFFT_REAL=float|double -DMIFFT_CHUNK=n; each object exports
// mifft_variants_<prec>_<chunk>().
#include "registry.hpp"

#ifndef MIFFT_REAL
#error "MIFFT_REAL must be float or double"
#endif
#ifndef MIFFT_CHUNK
#error "MIFFT_CHUNK must be set"
#endif

namespace mifft {

template <int L, int P, int E> constexpr Variant<MIFFT_REAL> make_variant()
{
    constexpr int TPL = threads_per_line(L, P, E);
    constexpr Factors f = factorize(L, P);
    Variant<MIFFT_REAL> v{};
    v.L = L;
    v.policy = P;
    v.emul = E;
    v.tpl = TPL;
    v.prefetch = strided_prefetches<MIFFT_REAL, L, P, TPL>() ? 1 : 0;
    v.poisson_B = poisson_tile_B<MIFFT_REAL, L, TPL>();
    v.nstages = f.n;
    for (int i = 0; i < f.n; ++i) v.radix[i] = f.r[i];
    v.contig = &k_contig<MIFFT_REAL, L, P, TPL, false>;
    v.contig_pack = &k_contig<MIFFT_REAL, L, P, TPL, true>;
    v.strided = &k_strided<MIFFT_REAL, L, P, TPL, 0>;
    v.strided_split = &k_strided<MIFFT_REAL, L, P, TPL, 1>;
    v.strided_osplit = &k_strided<MIFFT_REAL, L, P, TPL, 2>;
    v.r2c = &k_r2c_z<MIFFT_REAL, L, P, TPL>;
    v.c2r = &k_c2r_z<MIFFT_REAL, L, P, TPL>;
    v.poisson_x = &k_strided_poisson<MIFFT_REAL, L, P, TPL>;
    return v;
}

} // namespace mifft

#define MIFFT_CAT2(a, b) a##b
#define MIFFT_CAT(a, b) MIFFT_CAT2(a, b)
#define MIFFT_LEN(L, P, E) mifft::make_variant<L, P, E>(),

static const mifft::Variant<MIFFT_REAL> g_table[] = {
#include "variant_list.inc"
};

extern "C" const void* MIFFT_CAT(MIFFT_CAT(MIFFT_CAT(mifft_variants_, MIFFT_REAL), _), MIFFT_CHUNK)(int* n)
{
    *n = (int)(sizeof(g_table) / sizeof(g_table[0]));
    return g_table;
}
