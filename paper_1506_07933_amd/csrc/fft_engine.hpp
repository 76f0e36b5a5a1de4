// fft_engine.hpp -- device building blocks of the local 1-D FFT passes.
//
// The local phases of the pencil 3-D FFT (AccFFT, Sec. 2, Algorithm 1) are
// batches of independent 1-D DFTs along one axis.  Each line is transformed
// here by a Stockham autosort FFT: for a line of length L = R_1 R_2 ... R_s,
// stage k (radix R, Ns = R_1 ... R_{k-1} already combined) takes butterfly j
// (0 <= j < L/R) from positions j + r L/R, multiplies element r by the
// twiddle w_L^{(j mod Ns) r L/(Ns R)} (w_L = exp(-2 pi i / L)), applies a
// radix-R DFT and writes element r to (j div Ns) Ns R + (j mod Ns) + r Ns.
// The first stage therefore reads, and the last stage writes, in natural
// order with unit stride across threads, so both global accesses coalesce;
// the stages in between exchange through LDS.
//
// A "context" object supplies the global load of the first stage, the store
// of the last stage, the LDS addressing and the synchronisation, so the same
// stage code serves the contiguous-axis, strided-axis, R2C, C2R and fused
// pack / unpack kernels.  Inverse transforms use conj(F(conj(x))), so only
// forward butterflies and forward twiddles exist.
//
// A context that sets kPrefetch holds the first stage's inputs in registers
// (loaded ahead of time) and is asked, right after the first stage has
// consumed them, to load the inputs of its next tile into the same
// registers, so those loads are in flight while the rest of the current
// tile is transformed and stored.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>
#include <type_traits>

namespace mifft {

// ------------------------------------------------------------------ complex

template <typename T> struct cplx_of;
template <> struct cplx_of<float> { using type = float2; };
template <> struct cplx_of<double> { using type = double2; };
template <typename T> using cx = typename cplx_of<T>::type;

template <typename V> __device__ __forceinline__ V cadd(V a, V b) { return V{a.x + b.x, a.y + b.y}; }
template <typename V> __device__ __forceinline__ V csub(V a, V b) { return V{a.x - b.x, a.y - b.y}; }
template <typename V> __device__ __forceinline__ V cmul(V a, V b)
{
    return V{a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x};
}
template <typename V> __device__ __forceinline__ V cconj(V a) { return V{a.x, -a.y}; }
// multiply by -i: (a + ib)(-i) = b - ia
template <typename V> __device__ __forceinline__ V cmul_negi(V a) { return V{a.y, -a.x}; }
template <typename V, typename S> __device__ __forceinline__ V cscale(V a, S s) { return V{a.x * s, a.y * s}; }

// ------------------------------------------------------- radix butterflies
// Forward DFTs of 2, 3, 4, 5 and 8 points, in place: X[k] = sum_n v[n] w^{nk},
// w = exp(-2 pi i / R).  The constants are cos / sin of multiples of 2 pi / R.

template <int R> struct Bfly;

template <> struct Bfly<2> {
    template <typename V> __device__ __forceinline__ static void fwd(V* v)
    {
        V a = v[0], b = v[1];
        v[0] = cadd(a, b);
        v[1] = csub(a, b);
    }
};

template <> struct Bfly<4> {
    template <typename V> __device__ __forceinline__ static void fwd(V* v)
    {
        V t0 = cadd(v[0], v[2]), t1 = csub(v[0], v[2]);
        V t2 = cadd(v[1], v[3]), t3 = cmul_negi(csub(v[1], v[3]));
        v[0] = cadd(t0, t2);
        v[2] = csub(t0, t2);
        v[1] = cadd(t1, t3);
        v[3] = csub(t1, t3);
    }
};

template <> struct Bfly<8> {
    template <typename V> __device__ __forceinline__ static void fwd(V* v)
    {
        using S = decltype(v[0].x);
        const S h = S(0.707106781186547524400844362104849039); // 1/sqrt(2)
        // even / odd 4-point DFTs
        V e[4] = {v[0], v[2], v[4], v[6]};
        V o[4] = {v[1], v[3], v[5], v[7]};
        Bfly<4>::fwd(e);
        Bfly<4>::fwd(o);
        // o[k] *= w8^k: w8 = (1 - i)/sqrt2, w8^2 = -i, w8^3 = -(1 + i)/sqrt2
        V o1 = V{(o[1].x + o[1].y) * h, (o[1].y - o[1].x) * h};
        V o2 = cmul_negi(o[2]);
        V o3 = V{(o[3].y - o[3].x) * h, -(o[3].x + o[3].y) * h};
        v[0] = cadd(e[0], o[0]);
        v[4] = csub(e[0], o[0]);
        v[1] = cadd(e[1], o1);
        v[5] = csub(e[1], o1);
        v[2] = cadd(e[2], o2);
        v[6] = csub(e[2], o2);
        v[3] = cadd(e[3], o3);
        v[7] = csub(e[3], o3);
    }
};

template <> struct Bfly<3> {
    template <typename V> __device__ __forceinline__ static void fwd(V* v)
    {
        using S = decltype(v[0].x);
        const S s3 = S(0.866025403784438646763723170752936183); // sin(2 pi/3)
        V s = cadd(v[1], v[2]);
        V d = csub(v[1], v[2]);
        V m = V{v[0].x - S(0.5) * s.x, v[0].y - S(0.5) * s.y};
        V r = V{s3 * d.y, -s3 * d.x}; // -i sin(2 pi/3) (v1 - v2)
        v[0] = cadd(v[0], s);
        v[1] = cadd(m, r);
        v[2] = csub(m, r);
    }
};

template <> struct Bfly<5> {
    template <typename V> __device__ __forceinline__ static void fwd(V* v)
    {
        using S = decltype(v[0].x);
        const S c1 = S(0.309016994374947424102293417182819059);  // cos(2 pi/5)
        const S c2 = S(-0.809016994374947424102293417182819059); // cos(4 pi/5)
        const S s1 = S(0.951056516295153572116439333379382143);  // sin(2 pi/5)
        const S s2 = S(0.587785252292473129168705954639072769);  // sin(4 pi/5)
        V a1 = cadd(v[1], v[4]), b1 = csub(v[1], v[4]);
        V a2 = cadd(v[2], v[3]), b2 = csub(v[2], v[3]);
        V p1 = V{v[0].x + c1 * a1.x + c2 * a2.x, v[0].y + c1 * a1.y + c2 * a2.y};
        V p2 = V{v[0].x + c2 * a1.x + c1 * a2.x, v[0].y + c2 * a1.y + c1 * a2.y};
        V q1 = V{s1 * b1.x + s2 * b2.x, s1 * b1.y + s2 * b2.y};
        V q2 = V{s2 * b1.x - s1 * b2.x, s2 * b1.y - s1 * b2.y};
        // -i q = (q.y, -q.x)
        v[0] = cadd(v[0], cadd(a1, a2));
        v[1] = V{p1.x + q1.y, p1.y - q1.x};
        v[4] = V{p1.x - q1.y, p1.y + q1.x};
        v[2] = V{p2.x + q2.y, p2.y - q2.x};
        v[3] = V{p2.x - q2.y, p2.y + q2.x};
    }
};

// ----------------------------------------------------------- factorisation
// Radix lists are fixed at compile time.  Policy 0: the power-of-two part as
// radix 8 (a remainder of 2^1 becomes one radix-2 stage, 2^4 k+1 becomes
// 8..8,4,4), then radix 5, then radix 3.  Policy 1: the same radices in
// reverse order.  Policy 2: radix 4 first (a remainder 2), then 5, then 3.

struct Factors {
    int n;
    int r[24];
};

constexpr Factors factorize(int L, int policy)
{
    Factors f{0, {}};
    int a = 0, b = 0, c = 0, m = L;
    while (m % 2 == 0) { m /= 2; ++a; }
    while (m % 3 == 0) { m /= 3; ++b; }
    while (m % 5 == 0) { m /= 5; ++c; }
    if (m != 1) return Factors{-1, {}};
    if (policy == 2) {
        for (int i = 0; i < a / 2; ++i) f.r[f.n++] = 4;
        if (a % 2) f.r[f.n++] = 2;
    } else {
        int e8 = a / 3, rem = a % 3;
        if (rem == 1 && e8 >= 1) {
            for (int i = 0; i < e8 - 1; ++i) f.r[f.n++] = 8;
            f.r[f.n++] = 4;
            f.r[f.n++] = 4;
        } else {
            for (int i = 0; i < e8; ++i) f.r[f.n++] = 8;
            if (rem == 2) f.r[f.n++] = 4;
            if (rem == 1) f.r[f.n++] = 2;
        }
    }
    for (int i = 0; i < c; ++i) f.r[f.n++] = 5;
    for (int i = 0; i < b; ++i) f.r[f.n++] = 3;
    if (policy == 1) {
        for (int i = 0; i < f.n / 2; ++i) {
            int t = f.r[i];
            f.r[i] = f.r[f.n - 1 - i];
            f.r[f.n - 1 - i] = t;
        }
    }
    return f;
}

constexpr int max_radix(int L, int policy)
{
    Factors f = factorize(L, policy);
    int m = 1;
    for (int i = 0; i < f.n; ++i) m = f.r[i] > m ? f.r[i] : m;
    return m;
}

// Threads per line: L / (largest radix * emul) when that divides, else
// L / largest radix; at least 1.
constexpr int threads_per_line(int L, int policy, int emul)
{
    int mr = max_radix(L, policy);
    if (L % (mr * emul) == 0 && L / (mr * emul) >= 1) return L / (mr * emul);
    return L / mr > 0 ? L / mr : 1;
}

// ---------------------------------------------------------- fast division
// q = floor(k / d) for 0 <= k < 2^16 and 1 <= d <= 2^16, as (k * ceil(2^32/d)) >> 32.
// The rounded-up reciprocal overshoots by less than k 2^-32 < 2^-16 <= 1/d,
// which is below the gap between k/d and the next integer, so q is exact.
struct FastDiv {
    uint32_t d;
    uint64_t magic;
};

__device__ __forceinline__ uint32_t fdiv(uint32_t k, FastDiv f)
{
    return (uint32_t)(((uint64_t)k * f.magic) >> 32);
}

// ---------------------------------------------------------------- stages

// Contexts that declare kPrefetch = true supply first_get(slot) and
// prefetch_next<L, TPL, R>() (see FirstStageShape).
template <typename C, typename = void> struct ctx_prefetches : std::false_type {};
template <typename C>
struct ctx_prefetches<C, std::void_t<decltype(C::kPrefetch)>> : std::integral_constant<bool, C::kPrefetch> {};
// Contexts that declare kRegOut = true take the last stage's results as
// final_put_slot(slot, idx, v), slot = i R + r numbered as in FirstStageShape
// (the last stage of a Stockham transform writes elements j + r L/R, the
// set the first stage of a transform with that radix first reads).
template <typename C, typename = void> struct ctx_reg_out : std::false_type {};
template <typename C>
struct ctx_reg_out<C, std::void_t<decltype(C::kRegOut)>> : std::integral_constant<bool, C::kRegOut> {};

// The first stage's input positions: thread t reads, for its butterflies
// i = 0 .. NB-1 (j = t + i TPL < L/R) and r = 0 .. R-1, element j + r L/R
// into register slot i R + r.  each() visits (slot, element) in that order.
template <int L, int TPL, int R> struct FirstStageShape {
    static constexpr int NBF = L / R;
    static constexpr int NB = (NBF + TPL - 1) / TPL;
    static constexpr bool EXACT = (NBF % TPL) == 0;
    static constexpr int SLOTS = NB * R;
    template <typename F> __device__ __forceinline__ static void each(int t, F&& f)
    {
#pragma unroll
        for (int i = 0; i < NB; ++i) {
            const int j = t + i * TPL;
            if (EXACT || j < NBF) {
#pragma unroll
                for (int r = 0; r < R; ++r) f(i * R + r, j + r * NBF);
            }
        }
    }
};

template <typename T, int L, int TPL, int Ns, bool FIRST, typename Ctx, int R, int... Rest>
struct Stage {
    __device__ __forceinline__ static void run(Ctx& c)
    {
        using V = cx<T>;
        constexpr int NBF = L / R;                // butterflies in this stage
        constexpr int NB = (NBF + TPL - 1) / TPL; // butterflies per thread
        constexpr bool EXACT = (NBF % TPL) == 0;
        constexpr bool LAST = sizeof...(Rest) == 0;
        constexpr bool PF = FIRST && ctx_prefetches<Ctx>::value;
        V v[NB][R];
#pragma unroll
        for (int i = 0; i < NB; ++i) {
            const int j = c.t + i * TPL;
            if (EXACT || j < NBF) {
#pragma unroll
                for (int r = 0; r < R; ++r) {
                    if constexpr (PF)
                        v[i][r] = c.first_get(i * R + r);
                    else if constexpr (FIRST)
                        v[i][r] = c.gload(j + r * NBF);
                    else
                        v[i][r] = c.lds_get(j + r * NBF);
                }
            }
        }
        if constexpr (PF) c.template prefetch_next<L, TPL, R>();
        if constexpr (!FIRST || Ctx::kSyncAfterFirstRead) c.sync();
#pragma unroll
        for (int i = 0; i < NB; ++i) {
            const int j = c.t + i * TPL;
            if (EXACT || j < NBF) {
                if constexpr (Ns > 1) {
                    constexpr int step = L / (Ns * R);
                    const int k = j % Ns;
#pragma unroll
                    for (int r = 1; r < R; ++r) v[i][r] = cmul(v[i][r], c.tw(k * r * step));
                }
                Bfly<R>::fwd(v[i]);
                if constexpr (LAST) {
#pragma unroll
                    for (int r = 0; r < R; ++r) {
                        if constexpr (ctx_reg_out<Ctx>::value)
                            c.final_put_slot(i * R + r, j + r * NBF, v[i][r]);
                        else
                            c.final_put(j + r * NBF, v[i][r]);
                    }
                } else {
                    const int base = (j / Ns) * Ns * R + (j % Ns);
#pragma unroll
                    for (int r = 0; r < R; ++r) c.lds_put(base + r * Ns, v[i][r]);
                }
            }
        }
        if constexpr (!LAST) {
            c.sync();
            Stage<T, L, TPL, Ns * R, false, Ctx, Rest...>::run(c);
        }
    }
};

template <int... R> struct RadixList {};
template <typename RLt> struct FirstRadix;
template <int R0, int... Rest> struct FirstRadix<RadixList<R0, Rest...>> {
    static constexpr int value = R0;
};
template <> struct FirstRadix<RadixList<>> {
    static constexpr int value = 1; // length 1: no stage
};
// The radices in reverse order (a Stockham transform may take its factors in
// any order).
template <typename A, typename B> struct RLConcat;
template <int... A, int... B> struct RLConcat<RadixList<A...>, RadixList<B...>> {
    using type = RadixList<A..., B...>;
};
template <typename RLt> struct ReverseRL;
template <> struct ReverseRL<RadixList<>> { using type = RadixList<>; };
template <int R0, int... Rest> struct ReverseRL<RadixList<R0, Rest...>> {
    using type = typename RLConcat<typename ReverseRL<RadixList<Rest...>>::type, RadixList<R0>>::type;
};


template <typename T, int L, int TPL, typename Ctx, typename RL> struct LineFFT;
template <typename T, int L, int TPL, typename Ctx, int... R>
struct LineFFT<T, L, TPL, Ctx, RadixList<R...>> {
    __device__ __forceinline__ static void run(Ctx& c) { Stage<T, L, TPL, 1, true, Ctx, R...>::run(c); }
};

// RadixList for (L, policy) built from the constexpr factorisation.
template <int L, int P, typename Seq> struct MakeRL;
template <int L, int P, int... K> struct MakeRL<L, P, std::integer_sequence<int, K...>> {
    using type = RadixList<factorize(L, P).r[K]...>;
};
template <int L, int P>
using radix_list_t = typename MakeRL<L, P, std::make_integer_sequence<int, factorize(L, P).n>>::type;

// Padded LDS index for a contiguous line: one spare slot every 8 elements
// spreads the stride-R writes of the early stages over the LDS banks.
__device__ __forceinline__ int lds_pad(int idx) { return idx + (idx >> 3); }
__host__ __device__ constexpr int lds_padded_len(int L) { return L + (L >> 3) + 1; }

__device__ __forceinline__ void wave_sync()
{
    // The lanes that exchange data are in one wavefront and LDS requests of a
    // wavefront are served in order, so only compiler reordering must be
    // prevented here.
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

} // namespace mifft
