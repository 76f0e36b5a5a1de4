// kernels.hpp -- the HIP kernels of the local FFT passes (templates).
//
// k_contig   batched 1-D FFTs along the contiguous axis (the z-pass,
//            Algorithm 1), several lines per workgroup.  With
//            OUT_PACK the stores go straight to the row all-to-all send
//            layout S[j][i0][i1][m] (Sec. 2: pack before the exchange).
// k_strided  batched 1-D FFTs along a strided axis (the y- and x-passes,
//            Algorithm 1).  A workgroup owns a tile of B
//            adjacent columns, so every global access of a line element is a
//            run of B contiguous complex values.  With SPLIT = 1 the loads
//            follow the unpack map of the receive layout (Sec. 2: unpack after
//            the exchange), which fuses the unpack into the y-pass; with
//            SPLIT = 2 the stores follow the pack map of a send layout split
//            along the transformed axis (the slab transpose of Algorithm 3),
//            which fuses that pack into the y-pass.
// k_r2c_z    real z-lines: n2 reals are read as n2/2 complex values, FFT'd,
//            and post-processed into the n2/2+1 outputs of the real DFT.
// k_c2r_z    the inverse: pre-processing of the n2/2+1 inputs (imaginary
//            parts of k2 = 0 and n2/2 discarded), half-length inverse FFT,
//            de-interleave into n2 reals.
#pragma once

#include "fft_engine.hpp"
#include "spectral.hpp"

namespace mifft {

// ------------------------------------------------------------- contexts

// Streaming (non-temporal) stores for the passes' outputs: the next pass
// reads them gigabytes later, so keeping them in the caches buys nothing.
#ifndef MIFFT_CONTIG_NT
#define MIFFT_CONTIG_NT 1
#endif
#ifndef MIFFT_STRIDED_NT
#define MIFFT_STRIDED_NT 1
#endif
template <typename T> struct nt2_of;
template <> struct nt2_of<float> { typedef float type __attribute__((ext_vector_type(2))); };
template <> struct nt2_of<double> { typedef double type __attribute__((ext_vector_type(2))); };
template <typename T> __device__ __forceinline__ void store_nt(cx<T>* p, cx<T> v)
{
    typedef typename nt2_of<T>::type N2;
    __builtin_nontemporal_store(N2{v.x, v.y}, reinterpret_cast<N2*>(p));
}
// Streaming loads for the C2C passes' inputs (each element is read once).  The
// real-data passes and the fused spectral x-pass keep cached loads: with
// streaming loads there the R2C y-pass after them and the FP64 Poisson solve
// ran slower (2.45 -> 2.51 ms), while the C2C 512^3 forward gained 0.7% and
// the 4-D case 2.3%.
#ifndef MIFFT_NT_LOADS
#define MIFFT_NT_LOADS 1
#endif
// The fused spectral x-pass hands its spectrum from the forward to the
// inverse transform through the LDS tile (1) instead of registers (0).
#ifndef MIFFT_POISSON_LDS_HANDOFF
#define MIFFT_POISSON_LDS_HANDOFF 0
#endif
template <typename T> __device__ __forceinline__ cx<T> load_in(const cx<T>* p)
{
    if constexpr (MIFFT_NT_LOADS) {
        typedef typename nt2_of<T>::type N2;
        const N2 r = __builtin_nontemporal_load(reinterpret_cast<const N2*>(p));
        return cx<T>{r.x, r.y};
    } else {
        return *p;
    }
}

template <typename T, bool WAVE_LOCAL, bool OUT_PACK> struct ContigCtx {
    using V = cx<T>;
    static constexpr bool kSyncAfterFirstRead = false;
    const V* __restrict__ in;
    V* __restrict__ out;
    V* lds;
    const V* twd; // twiddle table staged in LDS
    int t;
    bool valid;
    T sgn;           // +1 forward, -1 inverse (conjugate on load and store)
    FastDiv pm;      // pack: block length M
    long long pblk;  // pack: distance between send blocks

    __device__ __forceinline__ V gload(int idx) const
    {
        V v = valid ? load_in<T>(in + idx) : V{T(0), T(0)};
        v.y *= sgn;
        return v;
    }
    __device__ __forceinline__ V lds_get(int idx) const { return lds[lds_pad(idx)]; }
    __device__ __forceinline__ void lds_put(int idx, V v) { lds[lds_pad(idx)] = v; }
    __device__ __forceinline__ void final_put(int idx, V v)
    {
        if (!valid) return;
        v.y *= sgn;
        if constexpr (OUT_PACK) {
            uint32_t q = fdiv((uint32_t)idx, pm);
            out[(long long)q * pblk + (idx - (int)(q * pm.d))] = v;
        } else if constexpr (MIFFT_CONTIG_NT) {
            store_nt<T>(out + idx, v);
        } else {
            out[idx] = v;
        }
    }
    __device__ __forceinline__ V tw(int e) const { return twd[e]; }
    __device__ __forceinline__ void sync() const
    {
        if constexpr (WAVE_LOCAL)
            wave_sync();
        else
            __syncthreads();
    }
};

// A strided workgroup transforms one column tile after another (tile,
// tile + grid, ...).  With PF the first stage's inputs of the next tile are
// loaded into registers while the current tile finishes (kPrefetch); PF is
// used where those registers fit next to the transform's own.
template <typename T, int SPLIT, int SLOTS, bool PF> struct StridedCtx {
    using V = cx<T>;
    static constexpr bool kSyncAfterFirstRead = false;
    static constexpr bool kPrefetch = PF;
    const V* __restrict__ in;
    V* __restrict__ out;
    V* lds; // column c of the tile: element idx at lds[idx * B]
    const V* twd; // twiddle table staged in LDS
    int t;
    int B;
    bool valid;
    T sgn;
    long long es_in, es_out; // element strides
    // SPLIT: element y = q * split.d + rem of a line sits at q * s_hi + rem * es
    // (es_in for SPLIT = 1 on the load side, es_out for SPLIT = 2 on the store side)
    FastDiv split;
    bool nt; // streaming loads: the tiles cover whole, aligned 128-byte lines of the input
    long long s_hi;
    V pre[SLOTS];            // first-stage inputs of the current tile
    const V* nin;            // next tile: input column, and whether it is a real column
    bool nvalid;
    bool has_next;

    __device__ __forceinline__ V raw_load(const V* __restrict__ base, bool ok, int idx) const
    {
        V v{T(0), T(0)};
        if (ok) {
            const V* p;
            if constexpr (SPLIT == 1) {
                uint32_t q = fdiv((uint32_t)idx, split);
                p = base + (long long)q * s_hi + (long long)(idx - (int)(q * split.d)) * es_in;
            } else {
                p = base + (long long)idx * es_in;
            }
            v = nt ? load_in<T>(p) : *p;
        }
        return v;
    }
    __device__ __forceinline__ V gload(int idx) const
    {
        V v = raw_load(in, valid, idx);
        v.y *= sgn;
        return v;
    }
    template <int L, int TPL, int R> __device__ __forceinline__ void load_first(const V* base, bool ok)
    {
        using S = FirstStageShape<L, TPL, R>;
#pragma unroll
        for (int i = 0; i < S::NB; ++i) {
            const int j = t + i * TPL;
            if (S::EXACT || j < S::NBF) {
#pragma unroll
                for (int r = 0; r < R; ++r) pre[i * R + r] = raw_load(base, ok, j + r * S::NBF);
            }
        }
    }
    __device__ __forceinline__ V first_get(int slot) const
    {
        V v = pre[slot];
        v.y *= sgn;
        return v;
    }
    template <int L, int TPL, int R> __device__ __forceinline__ void prefetch_next()
    {
        if (has_next) load_first<L, TPL, R>(nin, nvalid);
    }
    __device__ __forceinline__ V lds_get(int idx) const { return lds[idx * B]; }
    __device__ __forceinline__ void lds_put(int idx, V v) { lds[idx * B] = v; }
    __device__ __forceinline__ void final_put(int idx, V v)
    {
        if (!valid) return;
        v.y *= sgn;
        long long o;
        if constexpr (SPLIT == 2) {
            uint32_t q = fdiv((uint32_t)idx, split);
            o = (long long)q * s_hi + (long long)(idx - (int)(q * split.d)) * es_out;
        } else {
            o = (long long)idx * es_out;
        }
        if constexpr (MIFFT_STRIDED_NT)
            store_nt<T>(out + o, v);
        else
            out[o] = v;
    }
    __device__ __forceinline__ V tw(int e) const { return twd[e]; }
    __device__ __forceinline__ void sync() const { __syncthreads(); }
};

// R2C z-line: reads complex pairs of the real line, leaves Z in LDS.
template <typename T, bool WAVE_LOCAL> struct R2CCtx {
    using V = cx<T>;
    static constexpr bool kSyncAfterFirstRead = false;
    const V* __restrict__ in;
    V* lds;
    const V* twd; // twiddle table staged in LDS
    int t;
    bool valid;
    __device__ __forceinline__ V gload(int idx) const { return valid ? in[idx] : V{T(0), T(0)}; }
    __device__ __forceinline__ V lds_get(int idx) const { return lds[lds_pad(idx)]; }
    __device__ __forceinline__ void lds_put(int idx, V v) { lds[lds_pad(idx)] = v; }
    __device__ __forceinline__ void final_put(int idx, V v) { lds[lds_pad(idx)] = v; }
    __device__ __forceinline__ V tw(int e) const { return twd[e]; }
    __device__ __forceinline__ void sync() const
    {
        if constexpr (WAVE_LOCAL)
            wave_sync();
        else
            __syncthreads();
    }
};

// C2R z-line: the first stage reads the pre-processed (and conjugated)
// half-length input from the line staged in LDS.
template <typename T, bool WAVE_LOCAL> struct C2RCtx {
    using V = cx<T>;
    static constexpr bool kSyncAfterFirstRead = true;
    V* __restrict__ out; // the n2 reals of the line, as n2/2 pairs
    bool nt;             // streaming stores
    V* lds;
    const V* twd;               // twiddles of the half length M, staged in LDS
    const V* __restrict__ twd2; // exp(-2 pi i k / n2), k = 0 .. M
    int t;
    int M;
    bool valid;

    __device__ __forceinline__ V gload(int k) const
    {
        V z;
        if (k == 0) {
            T a = lds[lds_pad(0)].x, b = lds[lds_pad(M)].x;
            z = V{a + b, a - b};
        } else {
            V a = lds[lds_pad(k)];
            V b = cconj(lds[lds_pad(M - k)]);
            V s = cadd(a, b);
            V d = cmul(csub(a, b), cconj(twd2[k])); // (a - b) exp(+2 pi i k / n2)
            z = V{s.x - d.y, s.y + d.x};            // s + i d
        }
        return cconj(z);
    }
    __device__ __forceinline__ V lds_get(int idx) const { return lds[lds_pad(idx)]; }
    __device__ __forceinline__ void lds_put(int idx, V v) { lds[lds_pad(idx)] = v; }
    __device__ __forceinline__ void final_put(int idx, V v)
    {
        if (!valid) return;
        if (nt)
            store_nt<T>(out + idx, cconj(v));
        else
            out[idx] = cconj(v);
    }
    __device__ __forceinline__ V tw(int e) const { return twd[e]; }
    __device__ __forceinline__ void sync() const
    {
        if constexpr (WAVE_LOCAL)
            wave_sync();
        else
            __syncthreads();
    }
};

// A length-1 "FFT" is the identity.
template <typename T, int TPL, typename Ctx> struct LineFFT<T, 1, TPL, Ctx, RadixList<>> {
    __device__ __forceinline__ static void run(Ctx& c)
    {
        cx<T> v{T(0), T(0)};
        if (c.t == 0) v = c.gload(0);
        if constexpr (Ctx::kSyncAfterFirstRead) c.sync();
        if (c.t == 0) c.final_put(0, v);
    }
};

template <int L, int P> struct RL { using type = radix_list_t<L, P>; };
template <int P> struct RL<1, P> { using type = RadixList<>; };

template <int L, int TPL> constexpr bool wave_local() { return TPL <= 64 && (64 % TPL) == 0; }

// ---------------------------------------------------------------- kernels

// Copy the twiddle table of a line length into LDS (after the data tile):
// the butterflies then read it through the LDS path instead of issuing
// gathers through the vector memory path next to the data loads.
template <typename T>
__device__ __forceinline__ cx<T>* stage_twiddles(const cx<T>* __restrict__ tw, int L, cx<T>* dst)
{
    for (int i = threadIdx.x; i < L; i += blockDim.x) dst[i] = tw[i];
    __syncthreads();
    return dst;
}

// Grouped launches: with gridDim.y > 1, blockIdx.y selects one of up to
// kMaxGroup transforms of the same shape, each with its own buffers (a batch
// runs each pass of all its transforms of one shape as one launch).
constexpr int kMaxGroup = 16;
template <typename T> struct GroupPtrs {
    const cx<T>* in[kMaxGroup];
    cx<T>* out[kMaxGroup];
};

// Line l of a batch sits at (l / ni) * s_o + (l % ni) * s_i on each side, so a
// pass can read lines in one order and write them in another (the lines
// themselves stay contiguous).
template <typename T> struct ContigArgs {
    const cx<T>* in;
    cx<T>* out;
    GroupPtrs<T> grp;
    const cx<T>* tw;
    int nlines;
    int lines_per_wg;
    T sgn;
    FastDiv pm;
    long long pblk;
    int ni;
    long long is_o, is_i, os_o, os_i;
};

template <typename T, int L, int P, int TPL, bool OUT_PACK>
__global__ __launch_bounds__(1024) void k_contig(ContigArgs<T> a)
{
    using V = cx<T>;
    constexpr bool WL = wave_local<L, TPL>();
    extern __shared__ unsigned char smem_raw[];
    V* smem = reinterpret_cast<V*>(smem_raw);
    const int tid = threadIdx.x;
    const int ln = tid / TPL;
    const long long line = (long long)blockIdx.x * a.lines_per_wg + ln;
    ContigCtx<T, WL, OUT_PACK> c;
    c.valid = line < a.nlines;
    const V* ain = a.in;
    V* aout = a.out;
    if (gridDim.y > 1) {
        ain = a.grp.in[blockIdx.y];
        aout = a.grp.out[blockIdx.y];
    }
    const long long lo = line / a.ni, li = line - lo * a.ni;
    c.in = ain + lo * a.is_o + li * a.is_i;
    c.out = aout + lo * a.os_o + li * a.os_i; // with OUT_PACK: the line's place in block 0
    c.lds = smem + ln * lds_padded_len(L);
    c.twd = stage_twiddles<T>(a.tw, L, smem + a.lines_per_wg * lds_padded_len(L));
    c.t = tid - ln * TPL;
    c.sgn = a.sgn;
    c.pm = a.pm;
    c.pblk = a.pblk;
    LineFFT<T, L, TPL, decltype(c), typename RL<L, P>::type>::run(c);
}

template <typename T> struct StridedArgs {
    const cx<T>* in;
    cx<T>* out;
    GroupPtrs<T> grp;
    const cx<T>* tw;
    int B;
    int log2B;
    int cols;            // columns per group
    int ntiles;
    int groups;
    int tpg;             // tiles per group; 0: tiles over the flattened (group, column) index
    long long gs_in, gs_out; // group strides
    long long es_in, es_out; // element strides
    T sgn;
    FastDiv split;
    long long s_hi;
    int nt_in; // streaming loads (the planner's choice: whole, aligned input lines)
    // Two-level group maps: with gdiv > 1 group g sits at
    // (g / gdiv) * gs + (g % gdiv) * gs2 on that side (a blocked layout whose
    // two block indices have unrelated strides), else at g * gs.
    int gdiv_in, gdiv_out;
    long long gs2_in, gs2_out;
};

// Whether the strided kernel of (T, L, policy, TPL) prefetches the next
// tile: only where the prefetched data (first-stage elements per thread)
// fits in 32 VGPRs next to the transform's own registers without spilling
// at 1024 threads per workgroup (FP32; FP64 variants run the plain tile loop).
template <typename T, int L, int P, int TPL> constexpr bool strided_prefetches()
{
    using S = FirstStageShape<L, TPL, FirstRadix<typename RL<L, P>::type>::value>;
    return sizeof(T) == 4 && L > 1 && S::SLOTS * sizeof(cx<T>) <= 128;
}

// Tiles either stay within a group (tpg tiles per group, the last one
// ragged when B does not divide cols) or, with tpg = 0, run over the
// flattened column index f = group * cols + column (tile t holds f = t B ...
// t B + B - 1, so a tile may span two groups): where one side has gs = cols
// (the standard layout) its rows are then contiguous and aligned even when
// cols is not a multiple of B (the 257 columns of a half spectrum).
// Workgroup b takes tiles b, b + grid, b + 2 grid, ... (the grid may be
// smaller than the number of tiles, never larger).
template <typename T, int L, int P, int TPL, int SPLIT>
__global__ __launch_bounds__(1024) void k_strided(StridedArgs<T> a)
{
    using V = cx<T>;
    using RLt = typename RL<L, P>::type;
    constexpr int R0 = FirstRadix<RLt>::value;
    using Shape = FirstStageShape<L, TPL, R0>;
    constexpr bool PF = strided_prefetches<T, L, P, TPL>();
    const int ntiles = a.ntiles;
    int tile = blockIdx.x;
    if (tile >= ntiles) return; // uniform: the whole workgroup leaves
    extern __shared__ unsigned char smem_raw[];
    V* smem = reinterpret_cast<V*>(smem_raw);
    const int tid = threadIdx.x;
    const int cc = tid & (a.B - 1);
    StridedCtx<T, SPLIT, Shape::SLOTS, PF> c;
    c.lds = smem + cc;
    c.twd = stage_twiddles<T>(a.tw, L, smem + a.B * L);
    c.t = tid >> a.log2B;
    c.B = a.B;
    c.sgn = a.sgn;
    c.es_in = a.es_in;
    c.es_out = a.es_out;
    c.split = a.split;
    c.s_hi = a.s_hi;
    c.nt = a.nt_in != 0;
    // (group, column) of this thread in a tile; false past the last column
    auto locate = [&](int tl, long long& in_off, long long& out_off) -> bool {
        unsigned g, col;
        if (a.tpg > 0) {
            g = (unsigned)tl / (unsigned)a.tpg;
            col = ((unsigned)tl - g * (unsigned)a.tpg) * (unsigned)a.B + (unsigned)cc;
            if (col >= (unsigned)a.cols) g = (unsigned)a.groups; // padding column of a ragged tile
        } else {
            const unsigned f = (unsigned)tl * (unsigned)a.B + (unsigned)cc;
            g = f / (unsigned)a.cols;
            col = f - g * (unsigned)a.cols;
        }
        auto goff = [](unsigned gg, int d, long long s1, long long s2) -> long long {
            if (d > 1) {
                const unsigned q = gg / (unsigned)d;
                return (long long)q * s1 + (long long)(gg - q * (unsigned)d) * s2;
            }
            return (long long)gg * s1;
        };
        in_off = goff(g, a.gdiv_in, a.gs_in, a.gs2_in) + col;
        out_off = goff(g, a.gdiv_out, a.gs_out, a.gs2_out) + col;
        return g < (unsigned)a.groups;
    };
    const V* ain = a.in;
    V* aout = a.out;
    if (gridDim.y > 1) {
        ain = a.grp.in[blockIdx.y];
        aout = a.grp.out[blockIdx.y];
    }
    long long io = 0, oo = 0;
    c.valid = locate(tile, io, oo);
    c.in = ain + io;
    c.out = aout + oo;
    if constexpr (PF) c.template load_first<L, TPL, R0>(c.in, c.valid);
    for (;;) {
        // Hide the strides' loop invariance: hoisting the per-element address
        // products out of the tile loop would hold them all in registers.
        asm volatile("" : "+v"(c.es_in), "+v"(c.es_out), "+v"(c.B), "+v"(c.t));
        const int next = tile + (int)gridDim.x;
        c.has_next = next < ntiles;
        long long nio = 0, noo = 0;
        c.nvalid = c.has_next ? locate(next, nio, noo) : false;
        c.nin = ain + nio;
        LineFFT<T, L, TPL, decltype(c), RLt>::run(c);
        if (!c.has_next) break;
        __syncthreads(); // the next tile's first stage overwrites the LDS tile
        tile = next;
        c.valid = c.nvalid;
        c.in = c.nin;
        c.out = aout + noo;
    }
}

// ------------------------------------------- fused spectral x-pass
// The middle of a spectral operator (Poisson solve, Laplacian, Helmholtz
// solve, a partial derivative): on every x-line (fixed k1, k2) of the half
// spectrum, the forward x-FFT, the multiplication by the operator's m(k)
// (spectral_mul, the same expression as the standalone multiply) and the
// inverse x-FFT, with the line kept in LDS in between: one read and one
// write of the spectrum instead of three of each.  Column col of group g is
// (k1, k2) = (g + col / nc, col % nc), which covers both the transposed
// intermediate (groups = k1, columns = k2) and the standard layout (one
// group, columns = k1 nc + k2).  src may equal data (in place); with acc the
// result is added to what data holds (a sum of operators, e.g. divergence).
template <typename T> struct PoissonXArgs {
    const cx<T>* src;
    cx<T>* data;
    const cx<T>* tw;
    int cols;
    int groups;
    int tpg; // as in StridedArgs
    long long gs, es;
    int n1, nc, n2;
    int op, acc;
    T scale, alpha;
    int k2_fixed; // >= 0: every column is (k1, k2) = (column, k2_fixed) (a single k2 plane, [x][k1])
};

// PHASE 0: the forward transform; the first stage reads global memory and
// the last stage writes its results (scaled, and conjugated for the
// inverse) back into the LDS tile -- safe, because every stage after the
// first synchronises between reading its inputs from the tile and writing.
// PHASE 1: the inverse transform (of the conjugate) reads the line from LDS
// and stores the conjugate of its result.  B (columns per tile) is a
// compile-time constant, so the LDS offsets of a thread's elements are
// constants from one base address.  With REG the spectrum passes from one
// transform to the other in registers: the forward's last stage leaves its
// results in mid[] and the inverse, whose radix order is the forward's
// reversed, takes its first stage's inputs from there (the same elements,
// in the same threads).
template <typename T, int PHASE, int B, int SLOTS = 1, bool REG = false> struct PoissonCtx {
    using V = cx<T>;
    static constexpr bool kSyncAfterFirstRead = PHASE == 1 && !REG; // the first stage reads the LDS tile
    static constexpr bool kRegOut = PHASE == 0 && REG;
    static constexpr bool kPrefetch = PHASE == 1 && REG;
    V mid[REG ? SLOTS : 1];
    const V* src;
    V* data;
    V* lds; // column c of the tile: element idx at lds[idx * B]
    const V* twd;
    int t;
    bool valid;
    long long es;
    // PHASE 0: the multiplier
    int n0, op;
    SpectralCol<T> col; // this column's share of the multiplier
    T scale, alpha;
    // PHASE 1
    bool acc;

    __device__ __forceinline__ V gload(int idx) const
    {
        if constexpr (PHASE == 0)
            return valid ? src[(long long)idx * es] : V{T(0), T(0)};
        else
            return lds[idx * B];
    }
    __device__ __forceinline__ V first_get(int slot) const { return mid[slot]; }
    template <int L, int TPL, int R> __device__ __forceinline__ void prefetch_next() {}
    __device__ __forceinline__ void final_put_slot(int slot, int idx, V v)
    {
        v = spectral_mul<T>(op, idx, n0, col, scale, alpha, v);
        v.y = -v.y;
        mid[slot] = v;
    }
    __device__ __forceinline__ V lds_get(int idx) const { return lds[idx * B]; }
    __device__ __forceinline__ void lds_put(int idx, V v) { lds[idx * B] = v; }
    __device__ __forceinline__ void final_put(int idx, V v)
    {
        if constexpr (PHASE == 0) {
            v = spectral_mul<T>(op, idx, n0, col, scale, alpha, v);
            v.y = -v.y; // the inverse runs as conj(F(conj(.)))
            lds[idx * B] = v;
        } else {
            if (!valid) return;
            v.y = -v.y;
            V* p = data + (long long)idx * es;
            if (acc) {
                const V o = *p;
                v.x += o.x;
                v.y += o.y;
            }
            *p = v;
        }
    }
    __device__ __forceinline__ V tw(int e) const { return twd[e]; }
    __device__ __forceinline__ void sync() const { __syncthreads(); }
};

// Tile shape of the fused spectral x-pass for (T, L, TPL).  A workgroup
// loads its tile, runs two transforms on it and stores it, so a CU whose
// only workgroup is in its transforms has no memory traffic; the tile is
// therefore the widest (at most 256-byte rows) that lets two workgroups
// share a CU's 160 KiB of LDS, and the kernel is compiled for the register
// budget of two resident workgroups.  Measured on the 512^3 FP32 solve's
// x-pass: 32 columns, one workgroup per CU, 355 us; 16 columns of 64
// threads each, two per CU, 266 us (FP64: 16 -> 8 columns, 609 -> 517 us).
template <typename T, int L, int TPL> constexpr int poisson_tile_B()
{
    int b = 256 / (int)sizeof(cx<T>);
    while (b > 1 && (b * TPL > 1024 || (size_t)(b + 1) * L * sizeof(cx<T>) > 80 * 1024)) b /= 2;
    return b;
}
// Waves per SIMD the register allocation must allow: two workgroups per CU
// (four SIMDs), at least four (the budget of a 1024-thread workgroup) and,
// in FP64, at most four (at 64 registers the FP64 972-point kernel spilled).
template <typename T, int L, int TPL> constexpr int poisson_waves()
{
    const int waves = (poisson_tile_B<T, L, TPL>() * TPL + 63) / 64;
    const int w = (2 * waves + 3) / 4;
    const int cap = sizeof(T) == 8 ? 4 : 8;
    return w < 4 ? 4 : (w > cap ? cap : w);
}

template <typename T, int L, int P, int TPL>
__global__ __launch_bounds__((poisson_tile_B<T, L, TPL>() * TPL),
                             (poisson_waves<T, L, TPL>())) void k_strided_poisson(PoissonXArgs<T> a)
{
    using V = cx<T>;
    using RLt = typename RL<L, P>::type;
    constexpr int B = poisson_tile_B<T, L, TPL>();
    extern __shared__ unsigned char smem_raw[];
    V* smem = reinterpret_cast<V*>(smem_raw);
    const int tid = threadIdx.x;
    const int cc = tid & (B - 1);
    const int t = tid / B;
    // tiles as in k_strided
    int g, col;
    if (a.tpg > 0) {
        g = (int)blockIdx.x / a.tpg;
        col = ((int)blockIdx.x - g * a.tpg) * B + cc;
        if (col >= a.cols) g = a.groups; // padding column of a ragged tile
    } else {
        const unsigned f = (unsigned)blockIdx.x * (unsigned)B + (unsigned)cc;
        g = (int)(f / (unsigned)a.cols);
        col = (int)(f - (unsigned)g * (unsigned)a.cols);
    }
    // the inverse takes the radices in reverse order, so that its first stage
    // reads the elements the forward's last stage leaves in each thread
    constexpr bool REG = L > 1 && !MIFFT_POISSON_LDS_HANDOFF;
    using RLi = typename ReverseRL<RLt>::type;
    using Shape = FirstStageShape<L, TPL, FirstRadix<RLi>::value>;
    const V* twd = stage_twiddles<T>(a.tw, L, smem + B * L);
    PoissonCtx<T, 0, B, Shape::SLOTS, REG> c0;
    c0.valid = g < a.groups;
    const long long off = (long long)g * a.gs + col;
    c0.src = a.src + off;
    c0.data = a.data + off;
    c0.lds = smem + cc;
    c0.twd = twd;
    c0.t = t;
    c0.es = a.es;
    c0.n0 = L;
    c0.op = a.op;
    c0.col = a.k2_fixed >= 0 ? spectral_col<T>(a.op, col, a.k2_fixed, a.n1, a.n2, a.scale)
                             : spectral_col<T>(a.op, g + col / a.nc, col % a.nc, a.n1, a.n2, a.scale);
    c0.scale = a.scale;
    c0.alpha = a.alpha;
    LineFFT<T, L, TPL, decltype(c0), RLt>::run(c0);
    // Without REG the multiplied spectrum of every column is in the tile.
    // With it, no barrier: the forward's last stage synchronised after its
    // LDS reads, so the inverse's first stage may write the tile.
    if constexpr (!REG) __syncthreads();
    PoissonCtx<T, 1, B, Shape::SLOTS, REG> c1;
    if constexpr (REG) {
#pragma unroll
        for (int s = 0; s < Shape::SLOTS; ++s) c1.mid[s] = c0.mid[s];
    }
    c1.valid = c0.valid;
    c1.acc = a.acc != 0;
    c1.data = c0.data;
    c1.lds = c0.lds;
    c1.twd = twd;
    c1.t = t;
    c1.es = a.es;
    LineFFT<T, L, TPL, decltype(c1), std::conditional_t<REG, RLi, RLt>>::run(c1);
}

// Lines are mapped as in ContigArgs; offsets count complex elements of the
// complex side and pairs of reals (complex-sized units) of the real side.
template <typename T> struct RealArgs {
    const void* in;
    void* out;
    const cx<T>* tw;  // half-length twiddles
    const cx<T>* tw2; // exp(-2 pi i k / n2)
    int nt_out;       // streaming stores of the outputs
    // With nyq set, element M = n2/2 of the complex side (the Nyquist plane)
    // is not in the line but at nyq[lo * nyq_o + li * nyq_i] (a plane of its own).
    cx<T>* nyq;
    long long nyq_o, nyq_i;
    int nlines;
    int lines_per_wg;
    int ni;
    long long is_o, is_i, os_o, os_i;
};

// L = M = n2 / 2.
template <typename T, int L, int P, int TPL>
__global__ __launch_bounds__(1024) void k_r2c_z(RealArgs<T> a)
{
    using V = cx<T>;
    constexpr bool WL = wave_local<L, TPL>();
    extern __shared__ unsigned char smem_raw[];
    V* smem = reinterpret_cast<V*>(smem_raw);
    const int tid = threadIdx.x;
    const int ln = tid / TPL;
    const long long line = (long long)blockIdx.x * a.lines_per_wg + ln;
    R2CCtx<T, WL> c;
    c.valid = line < a.nlines;
    const long long lo = line / a.ni, li = line - lo * a.ni;
    c.in = reinterpret_cast<const V*>(a.in) + lo * a.is_o + li * a.is_i;
    c.lds = smem + ln * lds_padded_len(L + 1);
    c.twd = stage_twiddles<T>(a.tw, L, smem + a.lines_per_wg * lds_padded_len(L + 1));
    c.t = tid - ln * TPL;
    LineFFT<T, L, TPL, decltype(c), typename RL<L, P>::type>::run(c);
    c.sync();
    if (!c.valid) return;
    // X[k] = (a + b)/2 - (i/2) w^k (a - b),  a = Z[k mod M], b = conj(Z[(M - k) mod M])
    V* out = reinterpret_cast<V*>(a.out) + lo * a.os_o + li * a.os_i;
    const T half = T(0.5);
    for (int k = c.t; k <= L; k += TPL) {
        V za = c.lds[lds_pad(k == L ? 0 : k)];
        V zb = cconj(c.lds[lds_pad(k == 0 ? 0 : L - k)]);
        V s = cadd(za, zb);
        V p = cmul(a.tw2[k], csub(za, zb));
        const V r{half * (s.x + p.y), half * (s.y - p.x)};
        if (k == L && a.nyq)
            a.nyq[lo * a.nyq_o + li * a.nyq_i] = r;
        else if (a.nt_out)
            store_nt<T>(out + k, r);
        else
            out[k] = r;
    }
}

template <typename T, int L, int P, int TPL>
__global__ __launch_bounds__(1024) void k_c2r_z(RealArgs<T> a)
{
    using V = cx<T>;
    constexpr bool WL = wave_local<L, TPL>();
    extern __shared__ unsigned char smem_raw[];
    V* smem = reinterpret_cast<V*>(smem_raw);
    const int tid = threadIdx.x;
    const int ln = tid / TPL;
    const long long line = (long long)blockIdx.x * a.lines_per_wg + ln;
    C2RCtx<T, WL> c;
    c.valid = line < a.nlines;
    const long long lo = line / a.ni, li = line - lo * a.ni;
    c.lds = smem + ln * lds_padded_len(L + 1);
    c.twd = stage_twiddles<T>(a.tw, L, smem + a.lines_per_wg * lds_padded_len(L + 1));
    c.twd2 = a.tw2;
    c.nt = a.nt_out != 0;
    c.t = tid - ln * TPL;
    c.M = L;
    c.out = reinterpret_cast<V*>(a.out) + lo * a.os_o + li * a.os_i;
    if (c.valid) {
        const V* in = reinterpret_cast<const V*>(a.in) + lo * a.is_o + li * a.is_i;
        // all loads of the line in flight before the first LDS store (512^3
        // Poisson solve FP32 1.25 -> 1.20 ms).  FP64 holds them as native
        // two-element vectors (an array of cx<double> here was kept in scratch
        // memory), FP32 as cx<float> (native float vectors were, for the
        // lengths with many elements per thread).
        typedef std::conditional_t<sizeof(T) == 8, typename nt2_of<T>::type, V> N2;
        constexpr int NK = (L + 1 + TPL - 1) / TPL;
        N2 v[NK];
#pragma unroll
        for (int i = 0; i < NK; ++i) {
            const int k = c.t + i * TPL;
            if (k <= L)
                v[i] = *reinterpret_cast<const N2*>((k == L && a.nyq) ? a.nyq + (lo * a.nyq_o + li * a.nyq_i)
                                                                      : in + k);
        }
#pragma unroll
        for (int i = 0; i < NK; ++i) {
            const int k = c.t + i * TPL;
            if (k <= L) c.lds[lds_pad(k)] = V{v[i].x, v[i].y};
        }
    }
    c.sync();
    LineFFT<T, L, TPL, decltype(c), typename RL<L, P>::type>::run(c);
}

} // namespace mifft
