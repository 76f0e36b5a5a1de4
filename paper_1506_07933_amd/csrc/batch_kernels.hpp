// batch_kernels.hpp -- one persistent launch for many 3-D transforms of
// uneven sizes.
//
// Every (transform, pass) of the batch is a run of work items; the items of
// all z-passes come first in the queue (stage 0), then all y-passes (stage
// 1), then all x-passes (stage 2).  Persistent workgroups take items from a
// device counter in queue order.  An item of a y- or x-pass first waits
// until every item of the same transform's previous pass has completed (a
// per-pass completion counter).
//
// Completions are published lazily: a workgroup collects the items it has
// finished in a short pending list and publishes them (one release of its
// stores, then one counter update per pass and one per stage) only before
// it waits for anything, when the stage of its next item differs from the
// pending one, when the list is full, after a set number of completions,
// and when it leaves.  On this chip an
// agent-scope release writes back the XCD's L2 and an acquire invalidates
// it, so doing both per item would dominate the run; batched, a workgroup
// publishes a few times per stage.  Acquires are likewise skipped for a
// dependency already acquired, and for every pass of a stage that was seen
// complete before the workgroup's last acquire.
//
// The queue always drains: an item only waits for items that sit earlier in
// the queue, taken by workgroups that are running; a workgroup publishes
// everything it holds before it waits, so a holder either publishes on its
// way to its next wait or keeps taking items until the queue is empty and
// leaves, publishing then.  Every wait is bounded as well: a wait that
// exceeds its bound raises an abort flag that makes every workgroup leave.
//
// Inside a z-item each wavefront transforms its own contiguous lines,
// synchronising only within the wavefront.  A y- or x-item is a run of
// column tiles that the whole workgroup transforms one after another: a
// tile is as many adjacent columns as the workgroup holds lines of that
// length (kBatchBlock / threads per line), so each row of a tile is one contiguous
// run of 64 bytes or more (narrow per-wavefront column tiles made the
// strided passes several times slower).  Lanes left over when the threads
// per line do not divide the wavefront or workgroup work on a private dummy
// line or column whose results are discarded.
#pragma once

#include <stddef.h>

#include "kernels.hpp"

namespace mifft {

constexpr int kBatchMax = 128;      // transforms per batch (pointer slots in the kernel args)
// threads per workgroup (8 wavefronts).  Measured on the 64-transform batch
// (untuned): 256 threads 1.27 ms, 512 threads 1.09 ms, 1024 threads 1.19 ms
// -- wider column tiles (512 / threads per line columns) read longer rows.
constexpr int kBatchBlock = 512;
constexpr int kBatchWaves = kBatchBlock / 64;
constexpr int kBatchStages = 3;     // z, y, x
constexpr int kBatchPend = 16;      // passes in a workgroup's pending completion list

// Build-time choices (measured): twiddle copies in LDS, next-sub-tile
// prefetch, waves per SIMD of the persistent kernel, streaming stores.
#ifndef MIFFT_BATCH_TWL
#define MIFFT_BATCH_TWL 1
#endif
#ifndef MIFFT_BATCH_PF
#define MIFFT_BATCH_PF 1
#endif
#ifndef MIFFT_BATCH_WPE
#define MIFFT_BATCH_WPE 4
#endif
#ifndef MIFFT_BATCH_NT
#define MIFFT_BATCH_NT 0
#endif

// Line lengths with a code path in the persistent kernel: every length up to
// 256 with prime factors 2, 3, 5 whose threads per line fit one wavefront.
#define MIFFT_BATCH_MENU(X)                                                                       \
    X(0, 2) X(1, 3) X(2, 4) X(3, 5) X(4, 6) X(5, 8) X(6, 9) X(7, 10) X(8, 12) X(9, 15) X(10, 16)  \
    X(11, 18) X(12, 20) X(13, 24) X(14, 25) X(15, 27) X(16, 30) X(17, 32) X(18, 36) X(19, 40)      \
    X(20, 45) X(21, 48) X(22, 50) X(23, 54) X(24, 60) X(25, 64) X(26, 72) X(27, 75) X(28, 80)      \
    X(29, 81) X(30, 90) X(31, 96) X(32, 100) X(33, 108) X(34, 120) X(35, 125) X(36, 128)           \
    X(37, 135) X(38, 144) X(39, 150) X(40, 160) X(41, 162) X(42, 180) X(43, 192) X(44, 200)        \
    X(45, 216) X(46, 225) X(47, 240) X(48, 250) X(49, 256)

// Code paths per length: variant 0 uses the radix order of policy 0 with
// one radix group per thread, 1 the radix-4-first order (policy 2), 2 two
// radix groups per thread.  A variant that would equal variant 0 for a
// length is not compiled (its code runs variant 0); the autotuner picks one
// per (stage, length).
constexpr int kBatchVariants = 3;
__host__ __device__ constexpr int batch_var_policy(int v) { return v == 1 ? 2 : 0; }
__host__ __device__ constexpr int batch_var_emul(int v) { return v == 2 ? 2 : 1; }
__host__ __device__ constexpr bool batch_var_distinct(int L, int v)
{
    if (v == 1) {
        const Factors a = factorize(L, 0), b = factorize(L, 2);
        if (a.n != b.n) return true;
        for (int i = 0; i < a.n; ++i)
            if (a.r[i] != b.r[i]) return true;
        return false;
    }
    if (v == 2) return threads_per_line(L, 0, 2) != threads_per_line(L, 0, 1);
    return v == 0;
}

struct BatchPass {
    int kind;     // 0: contiguous z-lines, 1: strided columns
    int code;     // kBatchVariants x menu index of the line length + variant
    int L;
    int tpl;      // threads per line
    int xform;    // transform index (pointer slot)
    int from_in;  // 1: read the transform's input, 0: work in place on its output
    long long units;     // lines (kind 0) or columns over all groups (kind 1)
    int per_wave;        // lines / columns per wavefront sub-tile
    int subtiles;        // wavefront sub-tiles of this pass
    int subtiles_per_group; // kind 1
    int sub_per_item;    // sub-tiles per queue item (a multiple of the waves per workgroup)
    int nitems;
    int item_start;      // first queue index of this pass
    int cols;            // kind 1: columns per group
    long long gs, es;    // kind 1: group and element strides
    int stage;           // 0 z, 1 y, 2 x (queue order)
    int dep;             // completion counter to wait for, -1: none
    int dep_target;      // items it must reach
    int dep_stage;       // stage of that pass
    int done;            // completion counter of this pass
    const void* tw;      // twiddles of length L
};

template <typename T> struct BatchArgs {
    const BatchPass* passes;
    const int* item_pass; // pass of every queue item
    int npass;
    int total_items;
    // [0] queue head, [1 + p] completion of pass p, [1 + npass] abort flag,
    // [2 + npass + s] completion of stage s
    int* counters;
    int stage_items[kBatchStages]; // items per stage
    unsigned spin_limit;           // bound on the polls of one wait
    int publish_every;             // publish at the latest after this many completions
    const cx<T>* in[kBatchMax];
    cx<T>* out[kBatchMax];
};

// Dynamic LDS of the persistent kernel.  The kernel hands its base to the
// per-length functions as an LDS-address-space pointer: referenced from a
// non-inlined function, the symbol itself would be located through a global
// offset table, a memory load (and a full wait on all outstanding loads) at
// every use.
extern __shared__ __attribute__((aligned(16))) unsigned char mifft_batch_lds[];
#define MIFFT_LDS __attribute__((address_space(3)))

// Pointers read from memory are generic; the wave contexts hold them as
// global (address space 1) pointers so the compiler emits global, not flat,
// accesses, and the pass table is read through the constant address space
// (scalar loads).
#define MIFFT_GLOBAL __attribute__((address_space(1)))
#define MIFFT_CONST __attribute__((address_space(4)))

// Wave-local contexts -----------------------------------------------------

// Native two-element vectors are copied across address spaces freely (HIP's
// float2 / double2 classes are not), so global data moves as these.
template <typename T> struct vec2_of;
template <> struct vec2_of<float> { typedef float type __attribute__((ext_vector_type(2))); };
template <> struct vec2_of<double> { typedef double type __attribute__((ext_vector_type(2))); };

// Wave-local context of one sub-tile: lines (KIND 0: element idx of a line
// at idx) or columns (KIND 1: element idx at idx * es).  The first stage's
// inputs are prefetched into registers (PF: the next sub-tile's are loaded
// while the current one finishes), and the twiddles are read from the
// wavefront's LDS copy (TWL) or from global memory.
template <typename T, int KIND, int SLOTS, bool PF, bool TWL, bool WG = false> struct WaveCtx {
    using V = cx<T>;
    typedef typename vec2_of<T>::type N2;
    typedef MIFFT_GLOBAL N2 GN2;
    static constexpr bool kSyncAfterFirstRead = false;
    static constexpr bool kPrefetch = PF;
    typedef MIFFT_LDS N2 LN2;
    const GN2* in;
    GN2* out;
    LN2* lds;
    const LN2* twl; // TWL: the twiddle copy in LDS
    const GN2* twg; // otherwise: the twiddles in global memory
    int t;
    int rs;         // KIND 1: LDS row stride (columns of the sub-tile + 1)
    bool valid;
    long long es;   // KIND 1: element stride
    V pre[SLOTS > 0 ? SLOTS : 1];
    const GN2* nin;
    bool nvalid;
    bool has_next;

    __device__ __forceinline__ V raw(const GN2* base, bool ok, int idx) const
    {
        N2 r = N2{T(0), T(0)};
        if (ok) r = KIND == 0 ? base[idx] : base[(long long)idx * es];
        return V{r.x, r.y};
    }
    __device__ __forceinline__ V gload(int idx) const { return raw(in, valid, idx); }
    template <int L, int TPL, int R> __device__ __forceinline__ void load_first(const GN2* base, bool ok)
    {
        using S = FirstStageShape<L, TPL, R>;
#pragma unroll
        for (int i = 0; i < S::NB; ++i) {
            const int j = t + i * TPL;
            if (S::EXACT || j < S::NBF) {
#pragma unroll
                for (int r = 0; r < R; ++r) pre[i * R + r] = raw(base, ok, j + r * S::NBF);
            }
        }
    }
    __device__ __forceinline__ V first_get(int slot) const { return pre[slot]; }
    template <int L, int TPL, int R> __device__ __forceinline__ void prefetch_next()
    {
        if (has_next) load_first<L, TPL, R>(nin, nvalid);
    }
    __device__ __forceinline__ V lds_get(int idx) const
    {
        const N2 r = KIND == 0 ? lds[lds_pad(idx)] : lds[idx * rs];
        return V{r.x, r.y};
    }
    __device__ __forceinline__ void lds_put(int idx, V v)
    {
        if constexpr (KIND == 0)
            lds[lds_pad(idx)] = N2{v.x, v.y};
        else
            lds[idx * rs] = N2{v.x, v.y};
    }
    __device__ __forceinline__ void final_put(int idx, V v)
    {
        if (!valid) return;
        if constexpr (MIFFT_BATCH_NT) {
            if constexpr (KIND == 0)
                __builtin_nontemporal_store(N2{v.x, v.y}, out + idx);
            else
                __builtin_nontemporal_store(N2{v.x, v.y}, out + (long long)idx * es);
        } else {
            if constexpr (KIND == 0)
                out[idx] = N2{v.x, v.y};
            else
                out[(long long)idx * es] = N2{v.x, v.y};
        }
    }
    __device__ __forceinline__ V tw(int e) const
    {
        if constexpr (TWL) {
            const N2 r = twl[e];
            return V{r.x, r.y};
        } else {
            N2 r = twg[e];
            return V{r.x, r.y};
        }
    }
    __device__ __forceinline__ void sync() const
    {
        if constexpr (WG)
            __syncthreads();
        else
            wave_sync();
    }
};

// FP32 items keep a copy of the twiddle table in LDS and prefetch the next
// sub-tile or tile where its first-stage elements fit in 32 VGPRs; FP64
// items read twiddles from global memory and do not prefetch (register and
// LDS budget).
template <typename T> constexpr bool batch_tw_in_lds() { return MIFFT_BATCH_TWL && sizeof(T) == 4; }
template <typename T, int L, int P, int E> constexpr bool batch_prefetches()
{
    using S = FirstStageShape<L, threads_per_line(L, P, E), FirstRadix<typename RL<L, P>::type>::value>;
    return MIFFT_BATCH_PF && sizeof(T) == 4 && S::SLOTS * sizeof(cx<T>) <= 128;
}

// Columns of a workgroup column tile of length L.
__host__ __device__ constexpr int batch_tile_cols(int tpl) { return kBatchBlock / tpl > 0 ? kBatchBlock / tpl : 1; }

// LDS (elements) of one wavefront's z sub-tile of length L (contiguous lines
// plus a dummy line, then, with tw_lds, the twiddle table) and of a
// workgroup column tile (columns plus a dummy column, then the table).
__host__ __device__ constexpr int batch_wave_tile(int L, int tpl)
{
    return (64 / tpl + (64 % tpl ? 1 : 0)) * lds_padded_len(L); // dummy line only with left-over lanes
}
__host__ __device__ constexpr int batch_wave_lds(int L, int tpl, bool tw_lds)
{
    return batch_wave_tile(L, tpl) + (tw_lds ? L : 0);
}
__host__ __device__ constexpr int batch_col_tile(int L, int tpl)
{
    return L * (batch_tile_cols(tpl) + (kBatchBlock % tpl ? 1 : 0)); // dummy column only with left-over threads
}
// Dynamic LDS (elements) of a workgroup for a pass of length L: the larger of
// the two uses, so one size serves both kinds.
__host__ __device__ constexpr int batch_lds_elems(int L, int tpl, bool tw_lds)
{
    const int z = kBatchWaves * batch_wave_lds(L, tpl, tw_lds);
    const int c = batch_col_tile(L, tpl) + (tw_lds ? L : 0);
    return z > c ? z : c;
}

// Scalar copy of the fields a sub-tile needs (every field is uniform).
struct PassU {
    int kind, per_wave, subtiles_per_group, cols;
    long long units, gs, es;
    const void* tw;
};

__device__ __forceinline__ long long rfl64(long long v)
{
    const int lo = __builtin_amdgcn_readfirstlane((int)(v & 0xffffffffll));
    const int hi = __builtin_amdgcn_readfirstlane((int)(v >> 32));
    return (long long)(((unsigned long long)(unsigned)hi << 32) | (unsigned)lo);
}

__device__ __forceinline__ PassU load_pass(const MIFFT_CONST BatchPass* p)
{
    PassU u;
    u.kind = __builtin_amdgcn_readfirstlane(p->kind);
    u.per_wave = __builtin_amdgcn_readfirstlane(p->per_wave);
    u.subtiles_per_group = __builtin_amdgcn_readfirstlane(p->subtiles_per_group);
    u.cols = __builtin_amdgcn_readfirstlane(p->cols);
    u.units = rfl64(p->units);
    u.gs = rfl64(p->gs);
    u.es = rfl64(p->es);
    u.tw = (const void*)rfl64((long long)p->tw);
    return u;
}

// One code path per (length, radix policy, radix groups per thread), kept
// out of line so each gets its own register allocation.  z: the wavefront's
// sub-tiles first + wave, first + wave + 4, ...; y / x: the workgroup's
// column tiles first, first + 1, ...
template <typename T, int L, int P, int E>
__device__ __noinline__ void batch_item(const BatchPass* pp, const cx<T>* src, cx<T>* dst, int first, int last,
                                        int wave, int lane, MIFFT_LDS typename vec2_of<T>::type* lds)
{
    using V = cx<T>;
    typedef typename vec2_of<T>::type N2;
    typedef MIFFT_GLOBAL N2 GV;
    constexpr int TPL = threads_per_line(L, P, E);
    using RLt = typename RL<L, P>::type;
    constexpr int R0 = FirstRadix<RLt>::value;
    constexpr bool PF = batch_prefetches<T, L, P, E>();
    constexpr bool TWL = batch_tw_in_lds<T>();
    constexpr int SLOTS = PF ? FirstStageShape<L, TPL, R0>::SLOTS : 0;
    const PassU p = load_pass((const MIFFT_CONST BatchPass*)pp);
    const GV* twg = (const GV*)p.tw;
    typedef MIFFT_LDS N2 LN2;
    if (p.kind == 0) {
        constexpr int per = 64 / TPL;
        int s = first + wave;
        if (s >= last) return;
        LN2* wlds = lds + wave * batch_wave_lds(L, TPL, TWL);
        LN2* twl = wlds + batch_wave_tile(L, TPL);
        if constexpr (TWL) {
            for (int i = lane; i < L; i += 64) twl[i] = twg[i];
            wave_sync();
        }
        const int ui = lane / TPL; // line of this lane within the sub-tile
        WaveCtx<T, 0, SLOTS, PF, TWL> c;
        c.lds = wlds + (ui < per ? ui : per) * lds_padded_len(L);
        c.twl = twl;
        c.twg = twg;
        c.t = lane - ui * TPL;
        auto locate = [&](int sub, long long& off) -> bool {
            const long long line = (long long)sub * per + ui;
            off = line * L;
            return ui < per && line < p.units;
        };
        long long off = 0;
        c.valid = locate(s, off);
        c.in = (const GV*)(src + off);
        c.out = (GV*)(dst + off);
        if constexpr (PF) c.template load_first<L, TPL, R0>(c.in, c.valid);
#pragma nounroll
        for (;;) {
            asm volatile("" : "+v"(c.t)); // keep per-element addressing inside the loop
            const int nx = s + kBatchWaves;
            c.has_next = nx < last;
            long long noff = 0;
            c.nvalid = c.has_next ? locate(nx, noff) : false;
            c.nin = (const GV*)(src + noff);
            LineFFT<T, L, TPL, decltype(c), RLt>::run(c);
            if (!c.has_next) break;
            wave_sync(); // the next sub-tile's first stage overwrites this wavefront's tile
            s = nx;
            c.valid = c.nvalid;
            c.in = c.nin;
            c.out = (GV*)(dst + noff);
        }
    } else {
        // column tile: BC adjacent columns, column index fastest across threads
        constexpr int BC = batch_tile_cols(TPL);
        const int tid = threadIdx.x;
        const bool act = tid < BC * TPL;
        const int col_in = act ? tid % BC : BC;                  // BC: the dummy column
        const int t = act ? tid / BC : (tid - BC * TPL) % TPL;
        LN2* twl = lds + batch_col_tile(L, TPL);
        if constexpr (TWL) {
            for (int i = tid; i < L; i += kBatchBlock) twl[i] = twg[i];
            __syncthreads();
        }
        WaveCtx<T, 1, SLOTS, PF, TWL, true> c;
        c.rs = BC + (kBatchBlock % TPL ? 1 : 0);
        c.lds = lds + col_in;
        c.twl = twl;
        c.twg = twg;
        c.t = t;
        c.es = p.es;
        auto locate = [&](int tile, long long& off) -> bool {
            const int g = tile / p.subtiles_per_group;
            const int col = (tile - g * p.subtiles_per_group) * BC + col_in;
            off = (long long)g * p.gs + col;
            return act && col < p.cols;
        };
        int s = first;
        long long off = 0;
        c.valid = locate(s, off);
        c.in = (const GV*)(src + off);
        c.out = (GV*)(dst + off);
        if constexpr (PF) c.template load_first<L, TPL, R0>(c.in, c.valid);
#pragma nounroll
        for (;;) {
            asm volatile("" : "+v"(c.t), "+v"(c.es), "+v"(c.rs));
            const int nx = s + 1;
            c.has_next = nx < last;
            long long noff = 0;
            c.nvalid = c.has_next ? locate(nx, noff) : false;
            c.nin = (const GV*)(src + noff);
            LineFFT<T, L, TPL, decltype(c), RLt>::run(c);
            if (!c.has_next) break;
            __syncthreads(); // the next tile's first stage overwrites the LDS tile
            s = nx;
            c.valid = c.nvalid;
            c.in = c.nin;
            c.out = (GV*)(dst + noff);
        }
    }
}

template <typename T, int L, int V>
__device__ __forceinline__ void batch_item_var(const BatchPass* p, const cx<T>* src, cx<T>* dst, int first,
                                               int last, int wave, int lane,
                                               MIFFT_LDS typename vec2_of<T>::type* lds)
{
    if constexpr (batch_var_distinct(L, V))
        batch_item<T, L, batch_var_policy(V), batch_var_emul(V)>(p, src, dst, first, last, wave, lane, lds);
    else
        batch_item<T, L, 0, 1>(p, src, dst, first, last, wave, lane, lds);
}

template <typename T>
__device__ __forceinline__ void batch_dispatch(int code, const BatchPass* p, const cx<T>* src, cx<T>* dst,
                                               int first, int last, int wave, int lane,
                                               MIFFT_LDS typename vec2_of<T>::type* lds)
{
    switch (code) {
#define MIFFT_BATCH_CASE(I, LEN)                                                                  \
    case kBatchVariants * I:                                                                      \
        batch_item_var<T, LEN, 0>(p, src, dst, first, last, wave, lane, lds);                    \
        break;                                                                                    \
    case kBatchVariants * I + 1:                                                                  \
        batch_item_var<T, LEN, 1>(p, src, dst, first, last, wave, lane, lds);                    \
        break;                                                                                    \
    case kBatchVariants * I + 2:                                                                  \
        batch_item_var<T, LEN, 2>(p, src, dst, first, last, wave, lane, lds);                    \
        break;
        MIFFT_BATCH_MENU(MIFFT_BATCH_CASE)
#undef MIFFT_BATCH_CASE
    default:
        break;
    }
}

// Take the next queue item (or the end of the queue once the abort flag is up).
__device__ __forceinline__ int batch_dequeue(int* head, int* abort_flag, int total)
{
    if (__hip_atomic_load(abort_flag, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT)) return total;
    return __hip_atomic_fetch_add(head, 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// The explicit wait after the release makes the L2 write-back complete
// before the counter updates: the compiler drops its own wait after the
// write-back when no other vector memory operation is outstanding.
__device__ __forceinline__ void batch_release_agent()
{
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "agent");
    asm volatile("s_waitcnt vmcnt(0)" ::: "memory");
}

// Publish the pending completions of this workgroup (all threads call it,
// under a uniform condition).  Every wavefront waits until its own stores
// have reached the L2; after the barrier thread 0 releases at agent scope
// once for the workgroup (one L2 write-back, not one per wavefront: at the
// stage boundaries every workgroup publishes at about the same time, and
// the write-backs queue up) and adds the counts.
__device__ __forceinline__ void batch_publish(int* pass_done, int* stage_done, int pend_stage, int* s_npend,
                                              const int* s_pend_ctr, const int* s_pend_n)
{
    asm volatile("s_waitcnt vmcnt(0)" ::: "memory");
    __syncthreads();
    if (threadIdx.x == 0) {
        batch_release_agent();
        int total = 0;
        for (int i = 0; i < *s_npend; ++i) {
            __hip_atomic_fetch_add(pass_done + s_pend_ctr[i], s_pend_n[i], __ATOMIC_RELAXED,
                                   __HIP_MEMORY_SCOPE_AGENT);
            total += s_pend_n[i];
        }
        __hip_atomic_fetch_add(stage_done + pend_stage, total, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        *s_npend = 0;
    }
    __syncthreads();
}

// Loop structure: every region that only thread 0 executes sits between
// two workgroup barriers, and the loop's back edge leaves from a barrier.
// With a thread-0 region at the end of one iteration and another at the
// start of the next, the compiler may merge them across the back edge and
// let the other lanes run the next iteration's barrier before thread 0 has
// published the next item.  Thread 0 prepares the next item at the end of
// the current one (take it from the queue, find its pass, decide whether
// the pending completions must be published and whether it needs an
// acquire) and hands the decisions to the other threads through LDS.
template <typename T> __global__ __launch_bounds__(kBatchBlock) __attribute__((amdgpu_waves_per_eu(MIFFT_BATCH_WPE))) void k_batch(BatchArgs<T> a)
{
    using V = cx<T>;
    __shared__ int s_item, s_pass, s_abort, s_flush, s_need, s_npend;
    __shared__ int s_pend_ctr[kBatchPend], s_pend_n[kBatchPend];
    const int tid = threadIdx.x, wave = tid >> 6, lane = tid & 63;
    int* head = a.counters;
    int* pass_done = a.counters + 1;
    int* abort_flag = a.counters + 1 + a.npass;
    int* stage_done = a.counters + 2 + a.npass;
    // LDS address of the dynamic LDS, made opaque so that the compiler does not
    // propagate the symbol into the per-length functions
    unsigned lds_base = (unsigned)(size_t)(MIFFT_LDS unsigned char*)mifft_batch_lds;
    asm volatile("" : "+s"(lds_base));
    // thread 0's bookkeeping (registers of thread 0 only)
    int pend_stage = -1; // stage of the pending completions
    int pend_items = 0;  // completions pending
    int acq_dep = -1;    // last dependency acquired after it had completed
    int acq_stages = 0;  // stages seen complete before an acquire (bit mask)
    // thread 0: take the next item and decide what must precede it
    auto prepare = [&]() {
        const int it = batch_dequeue(head, abort_flag, a.total_items);
        s_item = it;
        s_flush = 0;
        s_need = 0;
        if (it >= a.total_items) return;
        const int lo = a.item_pass[it];
        s_pass = lo;
        const BatchPass* q = a.passes + lo;
        const int dep = q->dep, done = q->done;
        const int need = dep >= 0 && dep != acq_dep && !((acq_stages >> q->dep_stage) & 1);
        const int ready =
            !need || __hip_atomic_load(pass_done + dep, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) >= q->dep_target;
        int listed = 0;
        for (int k = 0; k < s_npend; ++k) listed |= s_pend_ctr[k] == done;
        s_need = need;
        s_flush = s_npend > 0 && (!ready || q->stage != pend_stage || (s_npend == kBatchPend && !listed) ||
                                  pend_items >= a.publish_every);
        if (s_flush) pend_items = 0;
    };
    if (tid == 0) {
        s_abort = 0;
        s_npend = 0;
        prepare();
    }
    __syncthreads();
    for (int iter = 0;; ++iter) {
        // uniform across the workgroup: keep the pass lookup and the code
        // switch scalar
        const int item = __builtin_amdgcn_readfirstlane(s_item);
        if (item >= a.total_items) break;
        if (iter > a.total_items) { // can only happen if the queue logic is broken: leave
            if (tid == 0) __hip_atomic_store(abort_flag, 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            break;
        }
        const BatchPass* pp = a.passes + __builtin_amdgcn_readfirstlane(s_pass);
        const int code = __builtin_amdgcn_readfirstlane(pp->code);
        const int from_in = __builtin_amdgcn_readfirstlane(pp->from_in);
        const int xform = __builtin_amdgcn_readfirstlane(pp->xform);
        const int item_start = __builtin_amdgcn_readfirstlane(pp->item_start);
        const int spi = __builtin_amdgcn_readfirstlane(pp->sub_per_item);
        const int subtiles = __builtin_amdgcn_readfirstlane(pp->subtiles);
        // 1. publish
        if (__builtin_amdgcn_readfirstlane(s_flush)) batch_publish(pass_done, stage_done, pend_stage, &s_npend, s_pend_ctr, s_pend_n);
        // 2. wait for the dependency and acquire
        if (__builtin_amdgcn_readfirstlane(s_need)) {
            if (tid == 0) {
                const int dep = pp->dep, target = pp->dep_target, ds = pp->dep_stage;
                unsigned polls = 0;
                while (__hip_atomic_load(pass_done + dep, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) < target) {
                    if (++polls > a.spin_limit ||
                        __hip_atomic_load(abort_flag, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT)) {
                        __hip_atomic_store(abort_flag, 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
                        s_abort = 1;
                        break;
                    }
                    __builtin_amdgcn_s_sleep(4);
                }
                // read before the acquire: a stage complete now is covered by it
                const int st_items = ds == 0 ? a.stage_items[0] : (ds == 1 ? a.stage_items[1] : a.stage_items[2]);
                const int full =
                    __hip_atomic_load(stage_done + ds, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) >= st_items;
                __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
                acq_dep = dep;
                if (full) acq_stages |= 1 << ds;
            }
            __syncthreads();
            if (__builtin_amdgcn_readfirstlane(s_abort)) break;
        }
        // 3. the item.  The pointer slots are read straight from the
        // kernel-argument segment (a uniform, dynamically indexed load) so the
        // argument block is never copied to private memory.
        const char* ka = (const char*)__builtin_amdgcn_kernarg_segment_ptr();
        V* const* outs = reinterpret_cast<V* const*>(ka + offsetof(BatchArgs<T>, out));
        const V* const* ins = reinterpret_cast<const V* const*>(ka + offsetof(BatchArgs<T>, in));
        const V* src = from_in ? ins[xform] : outs[xform];
        V* dst = outs[xform];
        const int first = (item - item_start) * spi;
        const int last = first + spi < subtiles ? first + spi : subtiles;
        batch_dispatch<T>(code, pp, src, dst, first, last, wave, lane,
                          (MIFFT_LDS typename vec2_of<T>::type*)(size_t)lds_base);
        // 4. thread 0: note the completion, prepare the next item
        __syncthreads();
        if (tid == 0) {
            const int done = pp->done;
            int k = 0;
            while (k < s_npend && s_pend_ctr[k] != done) ++k;
            if (k == s_npend) {
                s_pend_ctr[k] = done;
                s_pend_n[k] = 0;
                s_npend = k + 1;
            }
            s_pend_n[k] += 1;
            pend_stage = pp->stage;
            ++pend_items;
            prepare();
        }
        __syncthreads(); // the next item is published
    }
    // publish what is left (the loop leaves right after a barrier)
    if (__builtin_amdgcn_readfirstlane(s_npend) > 0)
        batch_publish(pass_done, stage_done, pend_stage, &s_npend, s_pend_ctr, s_pend_n);
}

// Zero the queue head, the completion counters and the abort flag (a kernel,
// not a memset, so the reset can be captured in a graph).
template <typename T> __global__ void k_batch_reset(int* counters, int n)
{
    for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < n; i += gridDim.x * blockDim.x) counters[i] = 0;
}

} // namespace mifft
