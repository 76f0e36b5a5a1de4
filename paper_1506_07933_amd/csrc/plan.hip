// plan.hip -- pass lists and launch geometry of a 3-D transform.
//
// Forward (Algorithm 1, left column, at P0 = P1 = 1): z-pass on the
// contiguous axis, then the y-pass (stride n2c), then the x-pass (stride
// n1 n2c).  Inverse (right column): x-pass, y-pass, z-pass.  The first pass
// reads the caller's input; every later pass works in place on the output
// (or, for C2R, on the workspace, so the input is preserved).
#include <cstdio>
#include <algorithm>
#include <cstdlib>
#include <cstring>
#include <mutex>

#include "aux_kernels.hpp"
#include "plan.hpp"

extern "C" {
const void* mifft_variants_float_0(int*);
const void* mifft_variants_float_1(int*);
const void* mifft_variants_float_2(int*);
const void* mifft_variants_float_3(int*);
const void* mifft_variants_double_0(int*);
const void* mifft_variants_double_1(int*);
const void* mifft_variants_double_2(int*);
const void* mifft_variants_double_3(int*);
}

namespace mifft {

// ------------------------------------------------------------------ errors

static thread_local std::string g_last_error;

int set_error(int status, const char* fmt, ...)
{
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof(buf), fmt, ap);
    va_end(ap);
    g_last_error = buf;
    return status;
}

void clear_error() { g_last_error.clear(); }

const char* last_error_cstr() { return g_last_error.c_str(); }

// ---------------------------------------------------------- variant tables

template <typename T> struct Table {
    std::vector<Variant<T>> v;
};

static std::once_flag g_tables_once;
static Table<float> g_f32;
static Table<double> g_f64;

static void load_tables()
{
    typedef const void* (*Getter)(int*);
    const Getter f32[] = {mifft_variants_float_0, mifft_variants_float_1, mifft_variants_float_2,
                          mifft_variants_float_3};
    const Getter f64[] = {mifft_variants_double_0, mifft_variants_double_1,
                          mifft_variants_double_2, mifft_variants_double_3};
    for (Getter g : f32) {
        int n = 0;
        const Variant<float>* p = (const Variant<float>*)g(&n);
        g_f32.v.insert(g_f32.v.end(), p, p + n);
    }
    for (Getter g : f64) {
        int n = 0;
        const Variant<double>* p = (const Variant<double>*)g(&n);
        g_f64.v.insert(g_f64.v.end(), p, p + n);
    }
}

template <typename T> static const std::vector<Variant<T>>& table();
template <> const std::vector<Variant<float>>& table<float>()
{
    std::call_once(g_tables_once, load_tables);
    return g_f32.v;
}
template <> const std::vector<Variant<double>>& table<double>()
{
    std::call_once(g_tables_once, load_tables);
    return g_f64.v;
}

template <typename F> static auto with_table(int prec, F f)
{
    if (prec == MIFFT_FP64) return f(table<double>());
    return f(table<float>());
}

int variant_count(int prec)
{
    return with_table(prec, [](const auto& t) { return (int)t.size(); });
}
int variant_L(int prec, int i)
{
    return with_table(prec, [i](const auto& t) { return t[i].L; });
}
int variant_tpl(int prec, int i)
{
    return with_table(prec, [i](const auto& t) { return t[i].tpl; });
}
int variant_policy(int prec, int i)
{
    return with_table(prec, [i](const auto& t) { return t[i].policy; });
}
int variant_emul(int prec, int i)
{
    return with_table(prec, [i](const auto& t) { return t[i].emul; });
}
int variant_prefetch(int prec, int i)
{
    return with_table(prec, [i](const auto& t) { return t[i].prefetch; });
}

int variant_poisson_B(int prec, int i)
{
    return with_table(prec, [i](const auto& t) { return t[i].poisson_B; });
}

int variant_radices(int prec, int i, int* radix, int max)
{
    return with_table(prec, [&](const auto& t) {
        const int n = t[i].nstages;
        for (int k = 0; k < n && k < max; ++k) radix[k] = t[i].radix[k];
        return n;
    });
}

int find_variant(int prec, int L, int policy, int emul)
{
    return with_table(prec, [&](const auto& t) {
        for (size_t i = 0; i < t.size(); ++i)
            if (t[i].L == L && t[i].policy == policy && t[i].emul == emul) return (int)i;
        return -1;
    });
}

int default_variant(int prec, int L)
{
    int i = find_variant(prec, L, 0, 1);
    if (i >= 0) return i;
    return with_table(prec, [&](const auto& t) {
        for (size_t k = 0; k < t.size(); ++k)
            if (t[k].L == L) return (int)k;
        return -1;
    });
}

// Variant of a contiguous-line pass (z, and the half-length lines of R2C /
// C2R): FP32 lines of 64 and 128 points take the radix-4-first variant, 16 /
// 32 threads per line instead of 8 / 16 -- the tuner's choice on every grid
// measured (z-pass of 512 x 512 x 64: 50.1 -> 43.9 us; 512 x 512 x 128:
// 94.5 -> 89.5 us; the 128-point half lines of R2C 256^3: 25.8 -> 25.3 us).
int contig_variant(int prec, int L)
{
    if (prec == MIFFT_FP32 && (L == 64 || L == 128)) {
        const int v = find_variant(prec, L, 2, 1);
        if (v >= 0) return v;
    }
    return default_variant(prec, L);
}

bool supported_length(int L)
{
    if (L < 1 || L > 1024) return false;
    int m = L;
    for (int p : {2, 3, 5})
        while (m % p == 0) m /= p;
    return m == 1;
}

FastDiv make_fastdiv(uint32_t d)
{
    FastDiv f;
    f.d = d;
    f.magic = ((1ull << 32) + d - 1) / d;
    return f;
}

// ---------------------------------------------------------------- geometry

static const size_t kLdsBudget = 64 * 1024;
static const size_t kLdsMax = 160 * 1024;

void set_contig_geometry(Pass& p, int prec, int tpl, int L, long long nlines, int lds_len)
{
    const size_t esz = prec == MIFFT_FP64 ? 16 : 8;
    // ~128 threads per workgroup (several small workgroups per CU overlap their
    // load, exchange and store phases), and at least two lines: a workgroup of
    // one 128-thread line (1024-point lines) ran 25% slower than one of two
    int lpw = 128 / tpl;
    if (lpw < 2) lpw = 2;
    while (lpw > 1 && ((size_t)lpw * lds_len + L) * esz > kLdsBudget) lpw /= 2;
    // keep enough workgroups to fill the chip when the batch is small
    while (lpw > 1 && lpw * tpl > 64 && (nlines + lpw - 1) / lpw < 1024) lpw /= 2;
    p.L = L;
    p.nlines = nlines;
    p.lines_per_wg = lpw;
    p.grid = (unsigned)((nlines + lpw - 1) / lpw);
    p.block = (unsigned)(lpw * tpl);
    p.shmem = ((size_t)lpw * lds_len + L) * esz; // tiles + the staged twiddle table
    set_line_map(p, (int)(nlines > 0 ? nlines : 1), 0, L, 0, L);
}

void set_line_map(Pass& p, int ni, long long is_o, long long is_i, long long os_o, long long os_i)
{
    p.ni = ni;
    p.is_o = is_o;
    p.is_i = is_i;
    p.os_o = os_o;
    p.os_i = os_i;
}

static int ilog2(int v)
{
    int r = 0;
    while ((1 << r) < v) ++r;
    return r;
}

void set_strided_geometry(Pass& p, int prec, int tpl, int L, int cols, int groups, int forceB)
{
    const size_t esz = prec == MIFFT_FP64 ? 16 : 8;
    int B = 16;
    if (forceB > 0) {
        B = forceB;
        while (B > 1 && ((size_t)B * tpl > 1024 || (size_t)(B + 1) * L * esz > kLdsMax)) B /= 2;
        while (B * tpl < 256 && B < 64 && (size_t)(2 * B + 1) * L * esz <= kLdsBudget) B *= 2;
        int cp = 1 << ilog2(cols < 1 ? 1 : cols);
        if (cp < B) B = cp;
    } else {
        while (B * tpl < 256 && B < 64) B *= 2;
        while (B > 1 && ((size_t)B * tpl > 1024 || (size_t)(B + 1) * L * esz > kLdsBudget)) B /= 2;
        int cp = 1 << ilog2(cols < 1 ? 1 : cols);
        if (cp < B) B = cp;
    }
    p.L = L;
    p.B = B;
    p.log2B = ilog2(B);
    p.cols = cols;
    p.groups = groups;
    p.ntiles = (int)(((long long)groups * cols + B - 1) / B);
    p.grid = (unsigned)p.ntiles;
    p.block = (unsigned)(B * tpl);
    p.shmem = ((size_t)B * L + L) * esz; // tile + the staged twiddle table
}

// A column tile of exactly B columns (the fused spectral x-pass's kernel is
// compiled for one width; columns past the end of a group are idle).
void set_tile_width(Pass& p, int prec, int tpl, int B)
{
    const size_t esz = prec == MIFFT_FP64 ? 16 : 8;
    p.B = B;
    p.log2B = ilog2(B);
    p.ntiles = (int)(((long long)p.groups * p.cols + B - 1) / B);
    p.grid = (unsigned)p.ntiles;
    p.block = (unsigned)(B * tpl);
    p.shmem = ((size_t)B * p.L + p.L) * esz; // tile + the staged twiddle table
}

// ----------------------------------------------------------------- launch

// Kernels whose dynamic LDS exceeds the default 64 KiB limit are opted in
// once (gfx950 has 160 KiB of LDS per CU).
static std::mutex g_lds_mu;
static std::map<const void*, size_t> g_lds_set;

static void ensure_lds(const void* fn, size_t bytes)
{
    if (bytes <= 65536) return;
    std::lock_guard<std::mutex> g(g_lds_mu);
    size_t& cur = g_lds_set[fn];
    if (cur >= bytes) return;
    if (hipFuncSetAttribute(fn, hipFuncAttributeMaxDynamicSharedMemorySize, (int)bytes) == hipSuccess)
        cur = bytes;
}

void tile_pass(const Plan& plan, Pass& p)
{
    if (p.kind != P_STRIDED && p.kind != P_STRIDED_SPLIT && p.kind != P_STRIDED_OSPLIT &&
        p.kind != P_POISSON_X)
        return;
    // a split side is not contiguous across groups
    const bool flat = (p.kind != P_STRIDED_OSPLIT && p.gs_out == p.cols) ||
                      (p.kind != P_STRIDED_SPLIT && p.gs_in == p.cols);
    p.tpg = flat ? 0 : (p.cols + p.B - 1) / p.B;
    p.ntiles = flat ? (int)(((long long)p.groups * p.cols + p.B - 1) / p.B) : p.groups * p.tpg;
    // Streaming (non-temporal) loads pay where every tile reads whole, aligned
    // 128-byte lines; where a tile reads part of a line that the next tile
    // reads too (ragged or unaligned rows: the 257 columns of a half
    // spectrum), the line must stay cached (measured: R2C 512^3 y-pass 0.255
    // -> 0.278 ms with streaming loads, the C2C 512^3 y-pass 0.415 -> 0.411).
    {
        const long long a = 128 / (long long)plan.esz;
        bool ok = p.cols % p.B == 0 && p.es_in % a == 0 && (p.groups == 1 || p.gs_in % a == 0) &&
                  (p.gdiv_in <= 1 || p.gs2_in % a == 0);
        if (p.kind == P_STRIDED_SPLIT) ok = ok && p.blk % a == 0;
        p.nt_in = ok ? 1 : 0;
    }
    if (p.kind == P_POISSON_X)
        p.grid = (unsigned)p.ntiles; // one workgroup per tile
    else
        strided_grid(plan, p);
}

void tile_passes(Plan& plan)
{
    for (auto* list : {&plan.fwd, &plan.inv, &plan.poisson, &plan.fwd_ip, &plan.inv_ip})
        for (Pass& p : *list) tile_pass(plan, p);
    for (Pass* p : {&plan.py, &plan.py_split, &plan.sy, &plan.sy_pack, &plan.sx, &plan.sxi, &plan.syi,
                    &plan.syi_unpack})
        tile_pass(plan, *p);
}

void strided_grid(const Plan& plan, Pass& p)
{
    const long long ntiles = p.ntiles;
    p.grid = (unsigned)ntiles;
    if (const char* e = getenv("MIFFT_STRIDED_PERSIST"))
        if (atoi(e) == 0) return;
    if (p.vidx < 0 || !variant_prefetch(plan.prec, p.vidx)) return;
    int per_cu = 0;
    if (!plan.plan_only) {
        const void* fn = with_table(plan.prec, [&](const auto& t) {
            return reinterpret_cast<const void*>(p.kind == P_STRIDED_SPLIT    ? t[p.vidx].strided_split
                                                 : p.kind == P_STRIDED_OSPLIT ? t[p.vidx].strided_osplit
                                                                              : t[p.vidx].strided);
        });
        ensure_lds(fn, p.shmem);
        if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, fn, (int)p.block, p.shmem) != hipSuccess) {
            (void)hipGetLastError();
            per_cu = 0;
        }
    }
    if (per_cu <= 0) { // estimate from LDS and threads (no device)
        per_cu = (int)std::min<size_t>((size_t)160 * 1024 / std::max<size_t>(p.shmem, 1), 2048 / p.block);
        per_cu = std::max(per_cu, 1);
    }
    // Resident grid, balanced: every workgroup walks the same number of tiles
    // (rounds), so no round runs with a few workgroups while the rest of the
    // device idles -- e.g. the 1032 tiles of the 256^3 R2C x-pass: 344
    // workgroups of 3 tiles instead of 512 with 8 of them taking a third.
    const long long cap = (long long)plan.cus * per_cu;
    if (ntiles > cap) {
        const long long rounds = (ntiles + cap - 1) / cap;
        p.grid = (unsigned)((ntiles + rounds - 1) / rounds);
    }
}

// ng > 1 (contiguous and strided passes): one launch over ng transforms of
// the same shape, member i reading gsrc[i] and writing gdst[i] (blockIdx.y).
template <typename T>
static hipError_t launch_fft(const Pass& p, const void* src, void* dst, hipStream_t s, int ng = 1,
                             const void* const* gsrc = nullptr, void* const* gdst = nullptr, void* nyq = nullptr)
{
    const Variant<T>& v = table<T>()[p.vidx];
    using V = cx<T>;
    switch (p.kind) {
    case P_CONTIG:
    case P_CONTIG_PACK: {
        ContigArgs<T> a{};
        a.in = (const V*)src;
        a.out = (V*)dst;
        for (int i = 0; i < ng && ng > 1; ++i) {
            a.grp.in[i] = (const V*)gsrc[i];
            a.grp.out[i] = (V*)gdst[i];
        }
        a.tw = (const V*)p.tw;
        a.nlines = (int)p.nlines;
        a.lines_per_wg = p.lines_per_wg;
        a.sgn = (T)p.sgn;
        a.pm = p.fd;
        a.pblk = p.blk;
        a.ni = p.ni;
        a.is_o = p.is_o;
        a.is_i = p.is_i;
        a.os_o = p.os_o;
        a.os_i = p.os_i;
        auto fn = p.kind == P_CONTIG ? v.contig : v.contig_pack;
        ensure_lds(reinterpret_cast<const void*>(fn), p.shmem);
        hipLaunchKernelGGL(fn, dim3(p.grid, ng), dim3(p.block), p.shmem, s, a);
        break;
    }
    case P_STRIDED:
    case P_STRIDED_SPLIT:
    case P_STRIDED_OSPLIT: {
        StridedArgs<T> a{};
        a.in = (const V*)src;
        a.out = (V*)dst;
        for (int i = 0; i < ng && ng > 1; ++i) {
            a.grp.in[i] = (const V*)gsrc[i];
            a.grp.out[i] = (V*)gdst[i];
        }
        a.tw = (const V*)p.tw;
        a.B = p.B;
        a.log2B = p.log2B;
        a.cols = p.cols;
        a.ntiles = p.ntiles;
        a.groups = p.groups;
        a.tpg = p.tpg;
        a.gs_in = p.gs_in;
        a.gs_out = p.gs_out;
        a.es_in = p.es_in;
        a.es_out = p.es_out;
        a.sgn = (T)p.sgn;
        a.split = p.fd;
        a.s_hi = p.blk;
        a.nt_in = p.nt_in;
        a.gdiv_in = p.gdiv_in;
        a.gdiv_out = p.gdiv_out;
        a.gs2_in = p.gs2_in;
        a.gs2_out = p.gs2_out;
        auto fn = p.kind == P_STRIDED         ? v.strided
                  : p.kind == P_STRIDED_SPLIT ? v.strided_split
                                              : v.strided_osplit;
        ensure_lds(reinterpret_cast<const void*>(fn), p.shmem);
        // a grid capped at the resident capacity is shared by the members
        unsigned gx = p.grid;
        if (ng > 1 && (int)p.grid < p.ntiles) gx = std::max(1u, (p.grid + (unsigned)ng - 1) / (unsigned)ng);
        hipLaunchKernelGGL(fn, dim3(gx, ng), dim3(p.block), p.shmem, s, a);
        break;
    }
    case P_POISSON_X: {
        PoissonXArgs<T> a;
        a.src = (const V*)src;
        a.data = (V*)dst;
        a.tw = (const V*)p.tw;
        a.cols = p.cols;
        a.groups = p.groups;
        a.tpg = p.tpg;
        a.gs = p.gs_in;
        a.es = p.es_in;
        a.n1 = p.n1;
        a.nc = p.n2c;
        a.n2 = p.nz;
        a.op = p.op;
        a.acc = p.acc;
        a.scale = (T)p.scale;
        a.alpha = (T)p.alpha;
        a.k2_fixed = p.k2_fixed;
        ensure_lds(reinterpret_cast<const void*>(v.poisson_x), p.shmem);
        hipLaunchKernelGGL(v.poisson_x, dim3(p.grid), dim3(p.block), p.shmem, s, a);
        break;
    }
    case P_R2C:
    case P_C2R: {
        RealArgs<T> a;
        a.in = src;
        a.out = dst;
        a.tw = (const V*)p.tw;
        a.tw2 = (const V*)p.tw2;
        a.nt_out = p.nt_out;
        a.nyq = p.nyq_buf != B_NONE ? (V*)nyq : nullptr;
        a.nyq_o = p.nyq_o;
        a.nyq_i = p.nyq_i;
        a.nlines = (int)p.nlines;
        a.lines_per_wg = p.lines_per_wg;
        a.ni = p.ni;
        a.is_o = p.is_o;
        a.is_i = p.is_i;
        a.os_o = p.os_o;
        a.os_i = p.os_i;
        auto fn = p.kind == P_R2C ? v.r2c : v.c2r;
        ensure_lds(reinterpret_cast<const void*>(fn), p.shmem);
        hipLaunchKernelGGL(fn, dim3(p.grid), dim3(p.block), p.shmem, s, a);
        break;
    }
    case P_POISSON:
        return launch_spectral<T>((const V*)src, (V*)dst, p.n0, p.n1, p.n2c, p.nz, p.op, (T)p.scale, (T)p.alpha,
                                  p.acc, s);
    case P_PACK:
        return launch_pack<T>((const V*)src, (V*)dst, p.n0, p.n1, p.p1, p.M, s);
    case P_UNPACK:
        return launch_unpack<T>((const V*)src, (V*)dst, p.n0, p.n1, p.p1, p.M, s);
    case P_COPY:
        return launch_copy(src, dst, p.bytes, s);
    }
    return hipGetLastError();
}

hipError_t launch_pass_group(const Pass& p, int prec, int ng, const void* const* src, void* const* dst,
                             hipStream_t s)
{
    if (ng < 1 || ng > kMaxGroup || (p.kind != P_CONTIG && p.kind != P_STRIDED)) return hipErrorInvalidValue;
    if (prec == MIFFT_FP64) return launch_fft<double>(p, src[0], dst[0], s, ng, src, dst);
    return launch_fft<float>(p, src[0], dst[0], s, ng, src, dst);
}

hipError_t launch_pass(const Pass& p, int prec, const void* src, void* dst, hipStream_t s, void* nyq)
{
    if (prec == MIFFT_FP64) return launch_fft<double>(p, src, dst, s, 1, nullptr, nullptr, nyq);
    return launch_fft<float>(p, src, dst, s, 1, nullptr, nullptr, nyq);
}

// --------------------------------------------------------------- twiddles

int get_twiddles(Plan& plan, int L, void** out)
{
    if (plan.plan_only) {
        *out = nullptr;
        return MIFFT_OK;
    }
    auto it = plan.twiddles.find(L);
    if (it != plan.twiddles.end()) {
        *out = it->second;
        return MIFFT_OK;
    }
    void* p = nullptr;
    hipError_t e = hipMalloc(&p, (size_t)L * plan.esz);
    if (e != hipSuccess) return set_error(MIFFT_ERR_NOMEM, "hipMalloc of %d twiddles: %s", L,
                                          hipGetErrorString(e));
    if (plan.prec == MIFFT_FP64)
        e = launch_twiddles<double>((cx<double>*)p, L, nullptr);
    else
        e = launch_twiddles<float>((cx<float>*)p, L, nullptr);
    if (e != hipSuccess) {
        hipFree(p);
        return set_error(MIFFT_ERR_DEVICE, "twiddle kernel: %s", hipGetErrorString(e));
    }
    plan.twiddles[L] = p;
    *out = p;
    return MIFFT_OK;
}

Plan::~Plan()
{
    for (SideLane& l : lane_pool) {
        if (l.s) hipStreamDestroy(l.s);
        if (l.fork) hipEventDestroy(l.fork);
        if (l.join) hipEventDestroy(l.join);
    }
    for (hipEvent_t e : prof_events) hipEventDestroy(e);
    for (auto& kv : twiddles) hipFree(kv.second);
    if (ws) hipFree(ws);
}

// ------------------------------------------------------------ pass builders

static int make_contig(Plan& plan, Pass& p, int L, long long nlines, int vidx)
{
    p.kind = P_CONTIG;
    p.vidx = vidx;
    int rc = get_twiddles(plan, L, (void**)&p.tw);
    if (rc) return rc;
    set_contig_geometry(p, plan.prec, variant_tpl(plan.prec, vidx), L, nlines, lds_padded_len(L));
    return MIFFT_OK;
}

// Column-tile shape of a strided pass: aim at 256-byte rows (B = 32 complex64
// or 16 complex128), the widest row that keeps the tile within 128 KiB of LDS
// and the workgroup within 1024 threads, trying the variants of L with the
// most threads per line first.  A group of more columns than that but at
// most twice as many (33 .. 64 complex64) is taken whole -- one tile per
// group, one contiguous block -- where that is not a multiple of the 256-byte
// row (e.g. the 51 of a half spectrum of 100: a full tile and a nearly empty
// one otherwise) or where the groups alone fill the device several times
// over (MIFFT_NARROW_TILES=0 keeps 256-byte rows, for comparison).
// Measured: R2C 256 x 256 x 100 forward 0.047 -> 0.042 ms; the 64-column
// axis of 512 x 256 x 128 x 64, 131072 groups: 3.42 -> 3.18 ms; with few
// groups (64^3) whole tiles were 7% slower.
static void choose_strided(const Plan& plan, int L, int cols, int groups, int* vidx, int* B)
{
    const int esz = (int)plan.esz;
    std::vector<int> cands;
    for (int i = 0; i < variant_count(plan.prec); ++i)
        if (variant_L(plan.prec, i) == L && variant_policy(plan.prec, i) == 0) cands.push_back(i);
    std::sort(cands.begin(), cands.end(), [&](int a, int b) {
        return variant_tpl(plan.prec, a) > variant_tpl(plan.prec, b);
    });
    int whole = 1;
    while (whole < cols) whole *= 2;
    bool narrow = true;
    if (const char* e = getenv("MIFFT_NARROW_TILES"))
        if (atoi(e) == 0) narrow = false;
    const bool many = (long long)groups >= 8LL * plan.cus;
    if (narrow && whole > 256 / esz && whole <= 512 / esz && (cols % (256 / esz) != 0 || many))
        for (int v : cands) {
            const int tpl = variant_tpl(plan.prec, v);
            if ((long long)tpl * whole <= 1024 && (size_t)(whole + 1) * L * esz <= 136 * 1024) {
                *vidx = v;
                *B = whole;
                return;
            }
        }
    for (int b = 256 / esz; b >= 1; b /= 2)
        for (int v : cands) {
            const int tpl = variant_tpl(plan.prec, v);
            if ((long long)tpl * b <= 1024 && (size_t)(b + 1) * L * esz <= 136 * 1024) {
                *vidx = v;
                *B = b;
                return;
            }
        }
    *vidx = default_variant(plan.prec, L);
    *B = 1;
}

static int make_strided(Plan& plan, Pass& p, int L, int cols, int groups, long long es,
                        long long gs, int vidx, int forceB)
{
    if (forceB == 0) choose_strided(plan, L, cols, groups, &vidx, &forceB);
    p.kind = P_STRIDED;
    p.vidx = vidx;
    int rc = get_twiddles(plan, L, (void**)&p.tw);
    if (rc) return rc;
    set_strided_geometry(p, plan.prec, variant_tpl(plan.prec, vidx), L, cols, groups, forceB);
    strided_grid(plan, p);
    p.es_in = p.es_out = es;
    p.gs_in = p.gs_out = gs;
    return MIFFT_OK;
}

static int make_real_z(Plan& plan, Pass& p, PassKind kind, long long nlines)
{
    const int M = plan.n2 / 2;
    const int vidx = contig_variant(plan.prec, M);
    if (vidx < 0) return set_error(MIFFT_ERR_UNSUPPORTED, "no kernel for half length %d", M);
    p.kind = kind;
    p.vidx = vidx;
    int rc = get_twiddles(plan, M, (void**)&p.tw);
    if (rc) return rc;
    rc = get_twiddles(plan, plan.n2, (void**)&p.tw2);
    if (rc) return rc;
    set_contig_geometry(p, plan.prec, variant_tpl(plan.prec, vidx), M, nlines, lds_padded_len(M + 1));
    // Streaming (non-temporal) stores where the output will not be read from
    // the caches anyway: an R2C spectrum larger than the 256 MB Infinity
    // Cache (a smaller one is read right away by the y-pass, from the cache:
    // 256^3 FP64 forward 0.181 ms cached, 0.200 streaming), and a C2R result
    // of 128 MiB or more (the end of the chain: 256^3 FP64 inverse 0.180 ->
    // 0.165 ms; FP32, 64 MiB, 0.103 -> 0.109 ms streaming; 512^3 Poisson
    // solve FP32 1.20 -> 1.17 ms, FP64 2.33 -> 2.25 ms with both streaming).
    {
        const double out_bytes = kind == P_R2C ? (double)nlines * (M + 1) * plan.esz : (double)nlines * M * plan.esz;
        p.nt_out = out_bytes > (kind == P_R2C ? 256.0 : 128.0) * 1024 * 1024 - 1 ? 1 : 0;
    }
    // complex side: lines of M + 1; real side: lines of M pairs
    const long long cl = M + 1, rl = M;
    if (kind == P_R2C)
        set_line_map(p, (int)p.nlines, 0, rl, 0, cl);
    else
        set_line_map(p, (int)p.nlines, 0, cl, 0, rl);
    return MIFFT_OK;
}

static int need_variant(Plan& plan, int L, int* v)
{
    *v = default_variant(plan.prec, L);
    if (*v < 0) return set_error(MIFFT_ERR_UNSUPPORTED, "no kernel for length %d", L);
    return MIFFT_OK;
}

// When the x-lines of the standard layout are far apart (stride n1 * n2c), a
// strided read of them is slow: every row of a column tile sits in a
// different translation page.  Strided writes with the same stride are
// cheap.  So the y-pass writes its output transposed, W[k1][x][k2] (stride
// n0 n2c between k1), and the x-pass then reads W with stride n2c and writes
// the standard layout; the inverse mirrors this.  This costs a workspace of
// the full (half) array.
static bool want_transposed(const Plan& plan, int nc)
{
    if (plan.n0 < 2 || plan.n1 < 2) return false;
    const size_t xstride = (size_t)plan.n1 * nc * plan.esz;
    return xstride >= (size_t)256 * 1024;
}

// Lines [line0, line0 + nlines) of a line pass as a pass of their own.
// Offsets are in bytes; one line-map unit is one complex element (or one pair
// of reals on the real side), i.e. `unit` bytes.
static Pass line_chunk(const Pass& p, long long line0, long long nlines, size_t unit)
{
    Pass q = p;
    q.nlines = nlines;
    q.grid = (unsigned)((nlines + q.lines_per_wg - 1) / q.lines_per_wg);
    if (p.ni >= p.nlines) { // contiguous line order: line l at l * s_i
        q.ni = (int)nlines;
        q.off_in = p.off_in + (long long)(line0 * p.is_i * (long long)unit);
        q.off_out = p.off_out + (long long)(line0 * p.os_i * (long long)unit);
    } else { // whole outer rows: line0 and nlines are multiples of ni
        const long long lo = line0 / p.ni;
        q.off_in = p.off_in + (long long)(lo * p.is_o * (long long)unit);
        q.off_out = p.off_out + (long long)(lo * p.os_o * (long long)unit);
    }
    return q;
}

static Pass group_chunk(const Plan& plan, const Pass& p, int g0, int ng, size_t esz)
{
    Pass q = p;
    q.groups = ng;
    q.ntiles = (int)(((long long)ng * q.cols + q.B - 1) / q.B);
    strided_grid(plan, q);
    q.off_in = p.off_in + (long long)g0 * p.gs_in * (long long)esz;
    q.off_out = p.off_out + (long long)g0 * p.gs_out * (long long)esz;
    return q;
}

// The transposed strategy's forward is z (lines of x-planes), y (tiles of
// x-planes, writing W[k1][x][k2]), x; the y-tiles of plane x only need that
// plane's z-lines.  Running z and y chunk by chunk, with chunks of about
// 128 MiB, lets each y-chunk read what its z-chunk just wrote while it still
// sits in the 256 MB Infinity Cache.  The inverse is chunked the same way
// over k1-planes: x^-1 (tiles of k1-planes of W), then z^-1 of those planes.
// MIFFT_CHUNK_MIB overrides the chunk size (0: no chunking).
void apply_chunking(Plan& plan)
{
    const bool real = plan.kind == MIFFT_R2C;
    const int nc = real ? plan.n2 / 2 + 1 : plan.n2;
    const size_t plane_bytes = (size_t)plan.n1 * nc * plan.esz;
    // opt-in: on the MI355X boxes measured so far the chunked order was slower
    size_t target = 0;
    if (const char* e = getenv("MIFFT_CHUNK_MIB")) target = (size_t)atol(e) << 20;
    if (target == 0) return;
    // balanced chunks of about `target` bytes; a single chunk is no pipeline
    const int k = (int)std::max<size_t>(1, ((size_t)plan.n0 * plane_bytes + target - 1) / target);
    if (k < 2) return;
    const int C = (plan.n0 + k - 1) / k;
    // forward: [z, y, x] with z over lines (x outer, y inner), y over x-groups
    if (plan.fwd.size() == 3) {
        const Pass z = plan.fwd[0], y = plan.fwd[1], x = plan.fwd[2];
        std::vector<Pass> f;
        for (int g0 = 0; g0 < plan.n0; g0 += C) {
            const int ng = std::min(C, plan.n0 - g0);
            f.push_back(line_chunk(z, (long long)g0 * plan.n1, (long long)ng * plan.n1, plan.esz));
            f.push_back(group_chunk(plan, y, g0, ng, plan.esz));
        }
        f.push_back(x);
        plan.fwd = f;
    }
    // inverse: [y^-1, x^-1, z^-1]; x^-1 over k1-groups of W, z^-1 over lines (k1 outer)
    if (plan.inv.size() == 3) {
        const Pass y = plan.inv[0], x = plan.inv[1], z = plan.inv[2];
        const size_t wplane = (size_t)plan.n0 * nc * plan.esz; // one k1-plane of W
        const int kz = (int)std::max<size_t>(1, ((size_t)plan.n1 * wplane + target - 1) / target);
        const int Cz = (plan.n1 + kz - 1) / kz;
        std::vector<Pass> v;
        v.push_back(y);
        for (int g0 = 0; g0 < plan.n1; g0 += Cz) {
            const int ng = std::min(Cz, plan.n1 - g0);
            v.push_back(group_chunk(plan, x, g0, ng, plan.esz));
            v.push_back(line_chunk(z, (long long)g0 * plan.n0, (long long)ng * plan.n0, plan.esz));
        }
        plan.inv = v;
    }
    plan.chunks = (plan.n0 + C - 1) / C;
}

// Variant of an L-point strided pass whose column tile is exactly B columns
// wide (within 1024 threads and 136 KiB of LDS), the one with the most
// threads per line; -1 if none.
static int strided_variant_for_B(const Plan& plan, int L, int B)
{
    int best = -1;
    for (int i = 0; i < variant_count(plan.prec); ++i) {
        if (variant_L(plan.prec, i) != L || variant_policy(plan.prec, i) != 0) continue;
        const int tpl = variant_tpl(plan.prec, i);
        if ((long long)tpl * B > 1024 || (size_t)(B + 1) * L * plan.esz > 136 * 1024) continue;
        if (best < 0 || tpl > variant_tpl(plan.prec, best)) best = i;
    }
    return best;
}

// Blocked schedule of an out-of-place C2C transform with the transposed
// intermediate.  A column tile reads its rows from one contiguous block
// when the pass before it stored them there, so each strided pass has one
// contiguous side instead of none (a copy with the y / x tile pattern of
// 512^3 ran at 5.3-5.4 TB/s with both sides strided, 5.7-5.8 TB/s with the
// reads contiguous).  With W the tile width (256-byte rows), z = zb W + zc
// and nb = n2 / W blocks:
//   z:  X[x][y][z]             -> T[x][zb][y][zc]  (stores through the pack map, M = W)
//   y:  tile (x, zb) of T      -> U[k1][zb][x][zc] (rows k1 n0 n2 apart)
//   x:  tile (k1, zb) of U     -> X[k0][k1][k2]    (rows k0 n1 n2 apart)
// Buffers: z IN -> OUT, y OUT -> WS, x WS -> OUT; the inverse runs the same
// three passes conjugated (the axes of a 3-D DFT may be transformed in any
// order).  In place (in == out) the z-pass would overwrite lines that are
// not read yet, so those calls run the transposed-schedule lists, kept in
// fwd_ip / inv_ip.  Returns whether the schedule applies.
static bool build_blocked(Plan& plan, int vz)
{
    const int n0 = plan.n0, n1 = plan.n1, n2 = plan.n2;
    int wbytes = 256;
    if (const char* e = getenv("MIFFT_BLOCK_BYTES")) wbytes = atoi(e);
    if (wbytes != 64 && wbytes != 128 && wbytes != 256 && wbytes != 512) return false;
    const int W = (int)(wbytes / (int)plan.esz);
    if (W < 1 || plan.kind != MIFFT_C2C || vz < 0 || n0 < 2 || n1 < 2 || n2 % W != 0) return false;
    // opt-in (MIFFT_BLOCKED=1): on the MI355X it measured the same as the
    // transposed schedule (512^3 complex64 forward 1.203 vs 1.199 ms)
    const char* be = getenv("MIFFT_BLOCKED");
    if (!be || atoi(be) == 0) return false;
    const int vy = strided_variant_for_B(plan, n1, W), vx = strided_variant_for_B(plan, n0, W);
    if (vy < 0 || vx < 0) return false;
    const int nb = n2 / W;
    const long long N = (long long)n0 * n1 * n2;
    if ((long long)nb * n0 >= (1LL << 31) || (long long)nb * n1 >= (1LL << 31) || N >= (1LL << 40)) return false;
    std::vector<Pass> lists[2];
    for (int d = 0; d < 2; ++d) {
        const int sgn = d == 0 ? +1 : -1;
        Pass z, y, x;
        if (make_contig(plan, z, n2, (long long)n0 * n1, vz)) return false;
        z.kind = P_CONTIG_PACK;
        z.fd = make_fastdiv((uint32_t)W);
        z.blk = (long long)n1 * W;
        set_line_map(z, n1, (long long)n1 * n2, n2, (long long)n1 * n2, W);
        z.sgn = sgn;
        z.tag = 0;
        z.src = B_IN;
        z.dst = B_OUT;
        // group g = x nb + zb: T block g at g n1 W; U row k1 at k1 n0 n2 + zb n0 W + x W
        if (make_strided(plan, y, n1, W, n0 * nb, W, (long long)n1 * W, vy, W) || y.B != W) return false;
        y.es_out = (long long)n0 * n2;
        y.gs_out = W;
        y.gs2_out = (long long)n0 * W;
        y.gdiv_out = nb;
        y.fixedB = W;
        y.sgn = sgn;
        y.tag = 1;
        y.src = B_OUT;
        y.dst = B_WS;
        // group g = k1 nb + zb: U block g at g n0 W; X row k0 at k0 n1 n2 + g W
        if (make_strided(plan, x, n0, W, n1 * nb, W, (long long)n0 * W, vx, W) || x.B != W) return false;
        x.es_out = (long long)n1 * n2;
        x.gs_out = W;
        x.fixedB = W;
        x.sgn = sgn;
        x.tag = 2;
        x.src = B_WS;
        x.dst = B_OUT;
        lists[d] = {z, y, x};
    }
    plan.fwd_ip = plan.fwd;
    plan.inv_ip = plan.inv;
    plan.fwd = lists[0];
    plan.inv = lists[1];
    plan.blocked = W;
    return true;
}

int build_plan(Plan& plan, unsigned /*flags*/)
{
    const bool real = plan.kind == MIFFT_R2C;
    const int n0 = plan.n0, n1 = plan.n1, n2 = plan.n2;
    const int nc = real ? n2 / 2 + 1 : n2;
    const long long plane = (long long)n1 * nc; // x stride of the standard layout
    const size_t half_bytes = (size_t)n0 * n1 * nc * plan.esz;
    const bool T = want_transposed(plan, nc);
    plan.transposed = T;
    // Rows of the internal transposed intermediate W are padded to a multiple
    // of 128 bytes (e.g. 257 -> 272 complex64 for the half spectrum of 512):
    // with an unaligned pitch every column tile straddles cache lines.
    int rw = (int)(128 / plan.esz);
    if (const char* e = getenv("MIFFT_PAD_ROWS")) // "0": unpadded rows (for comparison)
        if (atoi(e) == 0) rw = 1;
    const int ncw = (nc + rw - 1) / rw * rw;
    plan.ncw = ncw;
    const size_t w_bytes = (size_t)n0 * n1 * ncw * plan.esz;
    const bool has_z = real || n2 > 1;
    int rc, vy = -1, vx = -1, vz = -1;
    if (n1 > 1 && (rc = need_variant(plan, n1, &vy))) return rc;
    if (n0 > 1 && (rc = need_variant(plan, n0, &vx))) return rc;
    if (!real && n2 > 1 && (rc = need_variant(plan, n2, &vz))) return rc;
    if (vz >= 0) vz = contig_variant(plan.prec, n2);

    // ---------------- forward: z, y, x (Algorithm 1, left column)
    plan.fwd.clear();
    if (real) {
        Pass z;
        if ((rc = make_real_z(plan, z, P_R2C, (long long)plan.n0 * plan.n1))) return rc;
        z.tag = 0;
        plan.fwd.push_back(z);
    } else if (has_z) {
        Pass z;
        if ((rc = make_contig(plan, z, n2, (long long)n0 * n1, vz))) return rc;
        z.sgn = +1;
        z.tag = 0;
        plan.fwd.push_back(z);
    }
    if (n1 > 1) {
        Pass y;
        // tile = (x, B columns of k2); lines along y with stride nc
        if ((rc = make_strided(plan, y, n1, nc, n0, nc, plane, vy, 0))) return rc;
        if (T) {
            y.es_out = (long long)n0 * ncw; // W[k1][x][k2], rows of ncw
            y.gs_out = ncw;
        }
        y.sgn = +1;
        y.tag = 1;
        plan.fwd.push_back(y);
    }
    if (n0 > 1) {
        Pass x;
        if (T) {
            // tile = (k1, B columns of k2) of W; lines along x with stride ncw
            if ((rc = make_strided(plan, x, n0, nc, n1, ncw, (long long)n0 * ncw, vx, 0))) return rc;
            x.es_out = plane; // standard layout X[k0][k1][k2]
            x.gs_out = nc;
        } else {
            if ((rc = make_strided(plan, x, n0, (int)plane, 1, plane, 0, vx, 0))) return rc;
        }
        x.sgn = +1;
        x.tag = 2;
        plan.fwd.push_back(x);
    }
    if (plan.fwd.empty()) { // 1 x 1 x 1 C2C: the identity
        Pass c;
        c.kind = P_COPY;
        c.bytes = plan.esz;
        plan.fwd.push_back(c);
    }
    // buffers
    {
        auto& f = plan.fwd;
        for (size_t i = 0; i < f.size(); ++i) {
            f[i].src = i == 0 ? B_IN : B_OUT;
            f[i].dst = B_OUT;
        }
        if (T) {
            // ..., y: OUT (or IN) -> WS, x: WS -> OUT
            Pass& y = f[f.size() - 2];
            Pass& x = f[f.size() - 1];
            y.dst = B_WS;
            x.src = B_WS;
            x.dst = B_OUT;
        }
    }

    // ---------------- inverse
    // Standard layout: x^-1, y^-1, z^-1 (Algorithm 1, right column), in
    // place after the first pass (C2R keeps its input: workspace).
    // Transposed: y^-1 (input -> W, transposing), x^-1 in place on W, then
    // z^-1 reading the lines of W in transposed order.  The x and y inverses
    // act on different axes of the same array and commute exactly in exact
    // arithmetic, so the order only changes rounding.
    plan.inv.clear();
    if (T) {
        Pass y;
        if ((rc = make_strided(plan, y, n1, nc, n0, nc, plane, vy, 0))) return rc;
        y.es_out = (long long)n0 * ncw;
        y.gs_out = ncw;
        y.sgn = -1;
        y.tag = 1;
        y.src = B_IN;
        y.dst = B_WS;
        plan.inv.push_back(y);
        Pass x;
        if ((rc = make_strided(plan, x, n0, nc, n1, ncw, (long long)n0 * ncw, vx, 0))) return rc;
        x.sgn = -1;
        x.tag = 2;
        x.src = x.dst = B_WS;
        if (!has_z) { // no z-pass to undo the transposition: x^-1 writes the standard layout
            x.es_out = plane;
            x.gs_out = nc;
            x.dst = B_OUT;
        }
        plan.inv.push_back(x);
        if (has_z) {
            Pass z;
            // lines in the order of W (k1 outer, x inner): line (y, x) of W
            // is line (x, y) of the output, so a range of k1 planes is a
            // contiguous range of lines
            if (real) {
                if ((rc = make_real_z(plan, z, P_C2R, (long long)plan.n0 * plan.n1))) return rc;
                set_line_map(z, n0, (long long)n0 * ncw, (long long)ncw, (long long)(n2 / 2),
                             (long long)n1 * (n2 / 2));
            } else {
                if ((rc = make_contig(plan, z, n2, (long long)n0 * n1, vz))) return rc;
                set_line_map(z, n0, (long long)n0 * ncw, (long long)ncw, (long long)n2, (long long)n1 * n2);
                z.sgn = -1;
            }
            z.tag = 0;
            z.src = B_WS;
            z.dst = B_OUT;
            plan.inv.push_back(z);
        }
    } else {
        if (n0 > 1) {
            Pass x;
            if ((rc = make_strided(plan, x, n0, (int)plane, 1, plane, 0, vx, 0))) return rc;
            x.sgn = -1;
            x.tag = 2;
            plan.inv.push_back(x);
        }
        if (n1 > 1) {
            Pass y;
            if ((rc = make_strided(plan, y, n1, nc, n0, nc, plane, vy, 0))) return rc;
            y.sgn = -1;
            y.tag = 1;
            plan.inv.push_back(y);
        }
        if (real) {
            Pass z;
            if ((rc = make_real_z(plan, z, P_C2R, (long long)plan.n0 * plan.n1))) return rc;
            z.tag = 0;
            plan.inv.push_back(z);
        } else if (has_z) {
            Pass z;
            if ((rc = make_contig(plan, z, n2, (long long)n0 * n1, vz))) return rc;
            z.sgn = -1;
            z.tag = 0;
            plan.inv.push_back(z);
        }
        if (plan.inv.empty()) {
            Pass c;
            c.kind = P_COPY;
            c.bytes = plan.esz;
            plan.inv.push_back(c);
        }
        auto& v = plan.inv;
        if (!real) {
            for (size_t i = 0; i < v.size(); ++i) {
                v[i].src = i == 0 ? B_IN : B_OUT;
                v[i].dst = B_OUT;
            }
        } else {
            // complex passes input -> workspace -> workspace; C2R reads the
            // workspace (or the input when it is the only pass)
            for (size_t i = 0; i + 1 < v.size(); ++i) {
                v[i].src = i == 0 ? B_IN : B_WS;
                v[i].dst = B_WS;
            }
            v.back().src = v.size() == 1 ? B_IN : B_WS;
            v.back().dst = B_OUT;
        }
    }
    plan.fwd_ip.clear();
    plan.inv_ip.clear();
    plan.blocked = 0;
    const char* chunk_env = getenv("MIFFT_CHUNK_MIB");
    const bool chunked = chunk_env && atol(chunk_env) > 0;
    if (T && has_z && !chunked) build_blocked(plan, vz);
    if (T && has_z && !plan.blocked) apply_chunking(plan);
    bool inv_uses_ws = false, fwd_uses_ws = false;
    for (const Pass& q : plan.inv) inv_uses_ws |= (q.src == B_WS || q.dst == B_WS);
    for (const Pass& q : plan.fwd) fwd_uses_ws |= (q.src == B_WS || q.dst == B_WS);
    plan.ws_bytes = (inv_uses_ws || fwd_uses_ws) ? (T ? w_bytes : half_bytes) : 0;

    rebuild_poisson(plan);
    tile_passes(plan);
    if (plan.ws_bytes > plan.default_ws_bytes) plan.default_ws_bytes = plan.ws_bytes;
    return validate_extents(plan);
}

// ------------------------------------------------------------ extents
// Every pass's reads and writes, as the largest element offset (plus one)
// it touches in its source and destination buffers, checked against the
// buffers' sizes: a plan whose passes could reach past a buffer is an
// internal error, reported before anything is launched.  Units are
// complex elements (pairs of reals on the real side).

static long long line_map_extent(int ni, long long nlines, long long s_o, long long s_i, long long len)
{
    if (nlines <= 0) return 0;
    const long long inner = std::min<long long>(ni, nlines);
    return ((nlines - 1) / ni) * s_o + (inner - 1) * s_i + len;
}

Extent pass_extent(const Pass& p, size_t esz)
{
    Extent e{0, 0};
    const long long oi = p.off_in / (long long)esz, oo = p.off_out / (long long)esz;
    switch (p.kind) {
    case P_CONTIG:
        e.in = oi + line_map_extent(p.ni, p.nlines, p.is_o, p.is_i, p.L);
        e.out = oo + line_map_extent(p.ni, p.nlines, p.os_o, p.os_i, p.L);
        break;
    case P_CONTIG_PACK: {
        const long long M = p.fd.d;
        e.in = oi + line_map_extent(p.ni, p.nlines, p.is_o, p.is_i, p.L);
        e.out = oo + line_map_extent(p.ni, p.nlines, p.os_o, p.os_i, M) + (p.L / M - 1) * p.blk;
        break;
    }
    case P_STRIDED:
    case P_STRIDED_SPLIT:
    case P_STRIDED_OSPLIT:
    case P_POISSON_X: {
        const long long g = p.groups - 1, c = p.cols - 1, d = p.fd.d;
        // largest group offset on a side: g gs, or with a two-level map
        // (g / gdiv) gs + (g % gdiv) gs2 <= (g / gdiv) gs + (min(groups, gdiv) - 1) gs2
        auto gmax = [&](int gdiv, long long gs, long long gs2) -> long long {
            if (gdiv > 1) return (g / gdiv) * gs + (std::min<long long>(p.groups, gdiv) - 1) * gs2;
            return g * gs;
        };
        const long long gi = gmax(p.gdiv_in, p.gs_in, p.gs2_in), go = gmax(p.gdiv_out, p.gs_out, p.gs2_out);
        if (p.kind == P_STRIDED_SPLIT)
            e.in = oi + gi + c + (p.L / d - 1) * p.blk + (d - 1) * p.es_in + 1;
        else
            e.in = oi + gi + c + (long long)(p.L - 1) * p.es_in + 1;
        if (p.kind == P_STRIDED_OSPLIT)
            e.out = oo + go + c + (p.L / d - 1) * p.blk + (d - 1) * p.es_out + 1;
        else
            e.out = oo + go + c + (long long)(p.L - 1) * p.es_out + 1;
        break;
    }
    case P_R2C: // M pairs in, M + 1 complex out
        e.in = oi + line_map_extent(p.ni, p.nlines, p.is_o, p.is_i, p.L);
        e.out = oo + line_map_extent(p.ni, p.nlines, p.os_o, p.os_i, p.L + 1);
        break;
    case P_C2R:
        e.in = oi + line_map_extent(p.ni, p.nlines, p.is_o, p.is_i, p.L + 1);
        e.out = oo + line_map_extent(p.ni, p.nlines, p.os_o, p.os_i, p.L);
        break;
    case P_POISSON:
        e.in = e.out = (long long)p.n0 * p.n1 * p.n2c;
        break;
    default: // pack / unpack / copy: sized by their own plans
        break;
    }
    return e;
}

int validate_extents(const Plan& plan)
{
    if (plan.pencil) { // every buffer of a share holds (N0/p0) (N1/p1) N2 elements
        const long long n = (long long)(plan.n0 / plan.p0) * (plan.n1 / plan.p1) * plan.n2;
        const Pass* ps[] = {&plan.pz, &plan.pz_pack, &plan.py, &plan.py_split};
        const char* names[] = {"z", "z+pack", "y", "unpack+y"};
        for (int k = 0; k < 4; ++k) {
            const Extent e = pass_extent(*ps[k], plan.esz);
            if (e.in > n || e.out > n)
                return set_error(MIFFT_ERR_INVALID, "internal: pencil %s pass reaches %lld / %lld of %lld elements",
                                 names[k], e.in, e.out, n);
        }
        return MIFFT_OK;
    }
    if (plan.slab) { // every complex buffer holds (N0/p) N1 N2c elements; the real slab (N0/p) N1 N2/2 pairs
        const bool real = plan.kind == MIFFT_R2C;
        const long long nc = real ? plan.n2 / 2 + 1 : plan.n2;
        const long long n = (long long)(plan.n0 / plan.slab_p) * plan.n1 * nc;
        const long long r = real ? (long long)(plan.n0 / plan.slab_p) * plan.n1 * (plan.n2 / 2) : n;
        struct Item {
            const Pass* p;
            const char* name;
            long long in, out;
        } items[] = {{&plan.sz, "z", r, n},         {&plan.sy, "y", n, n},
                     {&plan.sy_pack, "y+pack", n, n}, {&plan.sx, "x", n, n},
                     {&plan.sxi, "x^-1", n, n},      {&plan.syi, "y^-1", n, n},
                     {&plan.syi_unpack, "unpack+y^-1", n, n}, {&plan.szi, "z^-1", n, r}};
        for (const Item& it : items) {
            const Extent e = pass_extent(*it.p, plan.esz);
            if (e.in > it.in || e.out > it.out)
                return set_error(MIFFT_ERR_INVALID,
                                 "internal: slab %s pass reaches %lld / %lld of %lld / %lld elements", it.name,
                                 e.in, e.out, it.in, it.out);
        }
        return MIFFT_OK;
    }
    const bool real = plan.kind == MIFFT_R2C;
    const long long esz = (long long)plan.esz;
    const long long N = (long long)plan.n0 * plan.n1 * plan.n2;
    const long long half = (long long)plan.n0 * plan.n1 * (plan.n2 / 2 + 1);
    const long long sig = real ? N / 2 : N;   // signal side, complex units
    const long long spec = real ? half : N;   // spectrum side
    const long long ws = (long long)(plan.ws_bytes / esz);
    const long long pw = (long long)(plan.poisson_ws_bytes / 2 / esz);
    struct List {
        const std::vector<Pass>* v;
        const char* name;
        long long in, out;
    } lists[] = {{&plan.fwd, "forward", sig, spec},         {&plan.inv, "inverse", spec, sig},
                 {&plan.poisson, "poisson", sig, sig},         {&plan.fwd_ip, "in-place forward", sig, spec},
                 {&plan.inv_ip, "in-place inverse", spec, sig}};
    for (const List& l : lists) {
        for (size_t k = 0; k < l.v->size(); ++k) {
            const Pass& p = (*l.v)[k];
            const Extent e = pass_extent(p, plan.esz);
            auto cap = [&](BufId b) -> long long {
                return b == B_IN ? l.in : b == B_OUT ? l.out : b == B_WS ? ws : (b == B_SEND || b == B_RECV) ? pw : 0;
            };
            if ((p.src != B_NONE && e.in > cap(p.src)) || (p.dst != B_NONE && e.out > cap(p.dst)))
                return set_error(MIFFT_ERR_INVALID,
                                 "internal: %s pass %zu reaches %lld / %lld elements of buffers holding %lld / %lld",
                                 l.name, k, e.in, e.out, cap(p.src), cap(p.dst));
            if (p.nyq_buf != B_NONE) { // the Nyquist plane of a real z-pass
                const long long lo = p.ni < p.nlines ? (p.nlines - 1) / p.ni : 0;
                const long long li = std::min<long long>(p.ni, p.nlines) - 1;
                const long long ne = p.nyq_off / esz + lo * p.nyq_o + li * p.nyq_i + 1;
                if (ne > cap(p.nyq_buf))
                    return set_error(MIFFT_ERR_INVALID, "internal: %s pass %zu reaches %lld of %lld Nyquist elements",
                                     l.name, k, ne, cap(p.nyq_buf));
            }
        }
    }
    return MIFFT_OK;
}

// Poisson (R2C plans).  Buffers: A = first half of the Poisson workspace,
// B = the second half.  With n0 > 1 the x-forward, the multiply and the
// x-inverse run as one fused pass:
//   transposed:  z (IN -> A), y (A -> B, W[k1][x][k2]), fused x (B),
//                y^-1 (B, in place on W), z^-1 (B -> OUT, W's line order);
//   standard:    z (IN -> A), y (A), fused x (A), y^-1 (A), z^-1 (A -> OUT).
// The inverses then run in the order x, y, z (the x and y inverses act on
// different axes and commute exactly in exact arithmetic).  Otherwise:
// forward into A, standalone multiply, inverse out of A.
void rebuild_poisson(Plan& plan)
{
    plan.poisson.clear();
    plan.poisson_ws_bytes = plan.spectral_ws_bytes = 0;
    plan.poisson_mul = -1;
    plan.poisson_mul_n = 1;
    if (plan.kind != MIFFT_R2C) return;
    const int nc = plan.n2 / 2 + 1;
    const size_t half_bytes = (size_t)plan.n0 * plan.n1 * nc * plan.esz;
    const double scale = 1.0 / ((double)plan.n0 * plan.n1 * plan.n2);
    auto remap = [](BufId b, BufId in, BufId out, BufId ws) {
        return b == B_IN ? in : b == B_OUT ? out : b == B_WS ? ws : b;
    };
    const Pass* fx = nullptr; // the forward x-pass
    for (const Pass& q : plan.fwd)
        if (q.tag == 2) fx = &q;
    const int vx = fx ? fx->vidx : -1;
    const char* unfused = getenv("MIFFT_POISSON_UNFUSED"); // "1": keep the standalone multiply
    if (plan.n0 > 1 && fx && !(unfused && atoi(unfused) != 0)) {
        const bool T = plan.transposed;
        const int M = plan.n2 / 2;
        // Nyquist plane on its own (transposed intermediate, rows of M whole
        // 128-byte lines): the z-pass stores the k2 = n2/2 plane as N[x][k1]
        // after W and the main passes transform exactly M columns (no ragged
        // 257th / 129th column); the plane's own chain -- y (contiguous lines
        // of N), fused x with k2 = n2/2, y^-1 -- runs beside them.
        bool split = T && plan.n1 > 1 && ((size_t)M * plan.esz) % 128 == 0;
        if (const char* e = getenv("MIFFT_POISSON_NYQ")) // "0": the 257th column in the rows (comparison)
            split = split && atoi(e) != 0;
        const int vyc = split ? contig_variant(plan.prec, plan.n1) : -1;
        if (split && vyc < 0) split = false;
        // both buffers are internal: with the transposed intermediate their
        // rows are padded to ncw (128-byte multiples), as W's are
        const int pitch = split ? M : T ? plan.ncw : nc;
        const int cols = split ? M : nc;
        const long long plane = (long long)plan.n1 * pitch;
        const long long noff = (long long)plan.n0 * plan.n1 * pitch * (long long)plan.esz; // N after W (bytes)
        const BufId D = T ? B_RECV : B_SEND; // where the spectrum sits from the y-pass on
        const long long lines = (long long)plan.n0 * plan.n1;
        int rc = 0;
        Pass z, yn; // (declared before the first jump to the fallback)
        // the z-passes over all lines (the forward / inverse lists may be chunked)
        if ((rc = make_real_z(plan, z, P_R2C, lines))) goto fallback;
        set_line_map(z, (int)z.nlines, 0, M, 0, pitch); // reals -> A, rows of `pitch`
        z.src = B_IN;
        z.dst = B_SEND;
        if (split) { // line l = x n1 + y: N[l]
            z.nyq_buf = D;
            z.nyq_off = noff;
            z.nyq_o = 0;
            z.nyq_i = 1;
            // the plane's passes touch only N: on large grids they run beside
            // the main chain (lane 1) from the z-pass on, and the C2R waits
            // for them.  Small solves keep them in line: there the fork and
            // join cost more than the plane's launches (served mix of 64^3 -
            // 512^3: median solve 0.164 -> 0.177 ms with them on a side stream;
            // 512^3 FP32 1.046 -> 1.026 ms).
            z.fork_after = (size_t)lines * M * plan.esz >= ((size_t)256 << 20);
        }
        plan.poisson.push_back(z);
        if (split) { // the Nyquist plane's y-lines: contiguous rows of N[x][k1]
            rc = make_contig(plan, yn, plan.n1, plan.n0, vyc);
            if (rc) goto fallback;
            yn.sgn = +1;
            yn.tag = 1;
            yn.src = yn.dst = D;
            yn.off_in = yn.off_out = noff;
            yn.lane = z.fork_after ? 1 : 0;
        }
        if (plan.n1 > 1) {
            Pass y;
            rc = make_strided(plan, y, plan.n1, cols, plan.n0, pitch, plane, plan.fwd[1].vidx, 0);
            if (rc) goto fallback;
            if (T) { // A -> W[k1][x][k2]
                y.es_out = (long long)plan.n0 * pitch;
                y.gs_out = pitch;
            }
            y.sgn = +1;
            y.tag = 1;
            y.src = B_SEND;
            y.dst = D;
            plan.poisson.push_back(y);
        }
        if (split) plan.poisson.push_back(yn);
        {
            // fused x, in place: the default variant of the length (the most
            // threads per line) and the tile width its kernel is compiled for
            Pass x;
            int vp = default_variant(plan.prec, plan.n0);
            if (vp < 0) vp = vx;
            if (T)
                rc = make_strided(plan, x, plan.n0, cols, plan.n1, pitch, (long long)plan.n0 * pitch, vp, 1);
            else
                rc = make_strided(plan, x, plan.n0, (int)plane, 1, plane, 0, vp, 1);
            if (rc) goto fallback;
            set_tile_width(x, plan.prec, variant_tpl(plan.prec, vp), variant_poisson_B(plan.prec, vp));
            x.kind = P_POISSON_X;
            x.n0 = plan.n0;
            x.n1 = plan.n1;
            x.n2c = pitch; // column -> (k1, k2) = (g + col / pitch, col % pitch)
            x.nz = plan.n2;
            x.scale = scale;
            x.tag = 2;
            x.src = x.dst = D;
            plan.poisson_mul = (int)plan.poisson.size();
            plan.poisson.push_back(x);
            if (split) { // the Nyquist plane: lines along x (stride n1), columns k1, k2 = n2/2
                Pass xn;
                rc = make_strided(plan, xn, plan.n0, plan.n1, 1, plan.n1, 0, vp, 1);
                if (rc) goto fallback;
                set_tile_width(xn, plan.prec, variant_tpl(plan.prec, vp), variant_poisson_B(plan.prec, vp));
                xn.kind = P_POISSON_X;
                xn.n0 = plan.n0;
                xn.n1 = plan.n1;
                xn.n2c = plan.n1;
                xn.nz = plan.n2;
                xn.k2_fixed = M;
                xn.scale = scale;
                xn.tag = 2;
                xn.src = xn.dst = D;
                xn.off_in = xn.off_out = noff;
                xn.lane = yn.lane;
                plan.poisson.push_back(xn);
                plan.poisson_mul_n = 2;
            }
        }
        if (split) {
            Pass yni = yn;
            yni.sgn = -1;
            plan.poisson.push_back(yni);
        }
        if (plan.n1 > 1) {
            Pass y;
            const int vy = plan.fwd[1].vidx;
            // transposed: lines along k1 of W (stride n0 pitch); groups = x, columns = k2
            rc = T ? make_strided(plan, y, plan.n1, cols, plan.n0, (long long)plan.n0 * pitch, pitch, vy, 0)
                   : make_strided(plan, y, plan.n1, cols, plan.n0, pitch, plane, vy, 0);
            if (rc) goto fallback;
            y.sgn = -1;
            y.tag = 1;
            y.src = y.dst = D;
            plan.poisson.push_back(y);
        }
        {
            Pass zi; // C2R; with the transposed intermediate, in W's line order
            if ((rc = make_real_z(plan, zi, P_C2R, lines))) goto fallback;
            if (!T)
                set_line_map(zi, (int)zi.nlines, 0, pitch, 0, M);
            else
                set_line_map(zi, plan.n0, (long long)plan.n0 * pitch, pitch, M, (long long)plan.n1 * M);
            zi.src = D;
            zi.dst = B_OUT;
            if (split) { // line (lo, li) = (y, x): N[x n1 + y]
                zi.nyq_buf = D;
                zi.nyq_off = noff;
                zi.nyq_o = 1;
                zi.nyq_i = plan.n1;
                zi.join_before = yn.lane == 1;
            }
            plan.poisson.push_back(zi);
        }
        // each half holds W (rows of `pitch`) and, split, the Nyquist plane
        plan.poisson_ws_bytes = 2 * (size_t)plan.n0 * plan.n1 * (pitch + (split ? 1 : 0)) * plan.esz;
        plan.spectral_ws_bytes = plan.poisson_ws_bytes / 2 * 3;
        if (plan.spectral_ws_bytes > plan.default_ws_bytes) plan.default_ws_bytes = plan.spectral_ws_bytes;
        return;
    fallback: // (only a failed twiddle allocation): the unfused solve
        plan.poisson.clear();
    }
    for (Pass q : plan.fwd) { // IN -> A (its OUT), workspace B
        q.src = remap(q.src, B_IN, B_SEND, B_RECV);
        q.dst = remap(q.dst, B_IN, B_SEND, B_RECV);
        plan.poisson.push_back(q);
    }
    Pass m;
    m.kind = P_POISSON;
    m.n0 = plan.n0;
    m.n1 = plan.n1;
    m.n2c = nc;
    m.nz = plan.n2;
    m.scale = scale;
    m.src = m.dst = B_SEND;
    plan.poisson_mul = (int)plan.poisson.size();
    plan.poisson.push_back(m);
    for (Pass q : plan.inv) { // A -> ... -> OUT, workspace B
        q.src = remap(q.src, B_SEND, B_OUT, B_RECV);
        q.dst = remap(q.dst, B_SEND, B_OUT, B_RECV);
        plan.poisson.push_back(q);
    }
    // the two halves are equal: A holds the standard layout, B the (padded)
    // transposed intermediate
    const size_t w_bytes = plan.transposed ? (size_t)plan.n0 * plan.n1 * plan.ncw * plan.esz : half_bytes;
    plan.poisson_ws_bytes = 2 * std::max(half_bytes, w_bytes);
    plan.spectral_ws_bytes = plan.poisson_ws_bytes / 2 * 3;
    if (plan.spectral_ws_bytes > plan.default_ws_bytes) plan.default_ws_bytes = plan.spectral_ws_bytes;
}

int build_pencil(Plan& plan, unsigned /*flags*/)
{
    const int n0l = plan.n0 / plan.p0, n1l = plan.n1 / plan.p1, N1 = plan.n1, N2 = plan.n2;
    const int M = N2 / plan.p1;
    const long long lines = (long long)n0l * n1l;
    int rc;
    const int vz = contig_variant(plan.prec, N2);
    const int vy = default_variant(plan.prec, N1);
    if (vz < 0 || vy < 0) return set_error(MIFFT_ERR_UNSUPPORTED, "no kernel for the share's axes");
    // Z in place on A
    if ((rc = make_contig(plan, plan.pz, N2, lines, vz))) return rc;
    plan.pz.src = plan.pz.dst = B_IN;
    // Z with the pack fused into its stores
    plan.pz_pack = plan.pz;
    plan.pz_pack.kind = P_CONTIG_PACK;
    plan.pz_pack.fd = make_fastdiv((uint32_t)M);
    plan.pz_pack.blk = lines * M;
    set_line_map(plan.pz_pack, (int)lines, 0, N2, 0, M); // line l at l M of each send block
    plan.pz_pack.src = B_IN;
    plan.pz_pack.dst = B_SEND;
    // standalone pack / unpack
    Pass pk;
    pk.kind = P_PACK;
    pk.n0 = n0l;
    pk.n1 = n1l;
    pk.p1 = plan.p1;
    pk.M = M;
    pk.src = B_IN;
    pk.dst = B_SEND;
    plan.pk = pk;
    Pass up = pk;
    up.kind = P_UNPACK;
    up.src = B_RECV;
    up.dst = B_OUT;
    plan.upk = up;
    // Y in place on B = [n0l][N1][M]
    if ((rc = make_strided(plan, plan.py, N1, M, n0l, M, (long long)N1 * M, vy, 0))) return rc;
    plan.py.src = plan.py.dst = B_OUT;
    // Y with the unpack fused into its loads: element y of column (i0, m) of
    // B lives at R[y / n1l][i0][y % n1l][m].
    plan.py_split = plan.py;
    plan.py_split.kind = P_STRIDED_SPLIT;
    plan.py_split.gs_in = (long long)n1l * M;
    plan.py_split.es_in = M;
    plan.py_split.fd = make_fastdiv((uint32_t)n1l);
    plan.py_split.blk = lines * M;
    plan.py_split.src = B_RECV;
    plan.py_split.dst = B_OUT;
    plan.pz.sgn = plan.pz_pack.sgn = plan.py.sgn = plan.py_split.sgn = +1;
    plan.pz.tag = plan.pz_pack.tag = 0;
    plan.py.tag = plan.py_split.tag = 1;
    plan.pk.tag = plan.upk.tag = 3;
    tile_passes(plan);
    return validate_extents(plan);
}


// One task's share of the slab decomposition (Algorithm 3) for p tasks: the
// spatial slab A[N0/p][N1][N2] and the spectral share X[N0][N1/p][N2c] hold
// the same number of complex elements, as do the send and receive buffers.
//   forward  z: in -> out (R2C for R2C plans); y: in place on out, or with
//            the pack fused, out -> send with element y of line (i0, k2) at
//            S[y / n1l][i0][y % n1l][k2]; x: recv -> out, the received blocks
//            stacked along x in sender order (no unpack needed).
//   inverse  x^-1: in -> send (block r = x rows r n0l ... is contiguous);
//            y^-1 with the unpack fused, recv -> send, element y of line
//            (i0, k2) read from R[y / n1l][i0][y % n1l][k2], or unpack then
//            y^-1 in place on send; z^-1: send -> out (C2R for R2C plans).
int build_slab(Plan& plan, unsigned /*flags*/)
{
    const int P = plan.slab_p;
    const bool real = plan.kind == MIFFT_R2C;
    const int N0 = plan.n0, N1 = plan.n1, N2 = plan.n2;
    const int n0l = N0 / P, n1l = N1 / P, nc = real ? N2 / 2 + 1 : N2;
    const long long lines = (long long)n0l * N1;
    const long long blk = (long long)n0l * n1l * nc; // one send block
    int rc, vx, vy, vz = -1;
    if ((rc = need_variant(plan, N0, &vx)) || (rc = need_variant(plan, N1, &vy))) return rc;
    if (!real && (rc = need_variant(plan, N2, &vz))) return rc;
    if (vz >= 0) vz = contig_variant(plan.prec, N2);
    // forward
    if (real)
        rc = make_real_z(plan, plan.sz, P_R2C, lines);
    else
        rc = make_contig(plan, plan.sz, N2, lines, vz);
    if (rc) return rc;
    plan.sz.src = B_IN;
    plan.sz.dst = B_OUT;
    if ((rc = make_strided(plan, plan.sy, N1, nc, n0l, nc, (long long)N1 * nc, vy, 0))) return rc;
    plan.sy.src = plan.sy.dst = B_OUT;
    plan.sy_pack = plan.sy;
    plan.sy_pack.kind = P_STRIDED_OSPLIT;
    plan.sy_pack.gs_out = (long long)n1l * nc;
    plan.sy_pack.es_out = nc;
    plan.sy_pack.fd = make_fastdiv((uint32_t)n1l);
    plan.sy_pack.blk = blk;
    plan.sy_pack.dst = B_SEND;
    // standalone pack: the pencil pack of [n0l][1][p * (n1l nc)], i.e. the y
    // axis split into p runs of n1l nc contiguous elements
    Pass pk;
    pk.kind = P_PACK;
    pk.n0 = n0l;
    pk.n1 = 1;
    pk.p1 = P;
    pk.M = n1l * nc;
    pk.src = B_OUT;
    pk.dst = B_SEND;
    plan.spk = pk;
    if ((rc = make_strided(plan, plan.sx, N0, n1l * nc, 1, (long long)n1l * nc, 0, vx, 0))) return rc;
    plan.sx.src = B_RECV;
    plan.sx.dst = B_OUT;
    plan.sz.sgn = plan.sy.sgn = plan.sy_pack.sgn = plan.sx.sgn = +1;
    // inverse
    plan.sxi = plan.sx;
    plan.sxi.src = B_IN;
    plan.sxi.dst = B_SEND;
    Pass up;
    up.kind = P_UNPACK; // A[i0][s n1l + i1][k2] = R[s][i0][i1][k2]: the pencil unpack
    up.n0 = n0l;
    up.n1 = n1l;
    up.p1 = P;
    up.M = nc;
    up.src = B_RECV;
    up.dst = B_SEND;
    plan.supk = up;
    plan.syi = plan.sy;
    plan.syi.src = plan.syi.dst = B_SEND;
    plan.syi_unpack = plan.syi;
    plan.syi_unpack.kind = P_STRIDED_SPLIT;
    plan.syi_unpack.gs_in = (long long)n1l * nc;
    plan.syi_unpack.es_in = nc;
    plan.syi_unpack.fd = make_fastdiv((uint32_t)n1l);
    plan.syi_unpack.blk = blk;
    plan.syi_unpack.src = B_RECV;
    if (real)
        rc = make_real_z(plan, plan.szi, P_C2R, lines);
    else
        rc = make_contig(plan, plan.szi, N2, lines, vz);
    if (rc) return rc;
    plan.szi.src = B_SEND;
    plan.szi.dst = B_OUT;
    plan.sxi.sgn = plan.syi.sgn = plan.syi_unpack.sgn = plan.szi.sgn = -1;
    plan.sz.tag = plan.szi.tag = 0;
    plan.sy.tag = plan.sy_pack.tag = plan.syi.tag = plan.syi_unpack.tag = 1;
    plan.sx.tag = plan.sxi.tag = 2;
    plan.spk.tag = plan.supk.tag = 3;
    tile_passes(plan);
    return validate_extents(plan);
}


// Arrays of rank d + 1 > 3 in C order (Algorithm 2 with every P_i = 1): the
// forward runs 1-D FFTs along the last axis (contiguous lines; R2C for real
// plans), then along axes d - 1, ..., 0, each a strided pass whose columns
// are the elements after the axis and whose groups are the index ranges
// before it; the inverse runs axes 0, ..., d - 1 and then the last axis
// (C2R for real plans).  Axes of length 1 are skipped.
//
// With a large stride of axis 0 (the rows of a column tile each in a
// different translation page) the 3-D plan's transposed intermediate is
// used with the axes after axis 1 flattened into one: the axis-1 pass
// writes W[k1][x0][rest] into the workspace and the axis-0 pass reads W with
// stride `rest` and writes the standard layout; the inverse runs axis 1
// (input -> W), axis 0 (W -> standard layout), then the others.  The C2R
// keeps its input, so a real plan's inverse runs its complex passes in the
// workspace (two spectra when W is used).
int build_nd(Plan& plan, unsigned /*flags*/)
{
    const std::vector<int>& d = plan.dims;
    const int r = (int)d.size();
    const bool real = plan.kind == MIFFT_R2C;
    const int nl = d[r - 1];
    const long long nc = real ? nl / 2 + 1 : nl;
    std::vector<long long> inner(r), outer(r);
    inner[r - 1] = 1;
    for (int i = r - 2; i >= 0; --i) inner[i] = inner[i + 1] * (i + 1 == r - 1 ? nc : d[i + 1]);
    outer[0] = 1;
    for (int i = 1; i < r; ++i) outer[i] = outer[i - 1] * d[i - 1];
    const long long lines = outer[r - 1];
    const size_t spec_bytes = (size_t)lines * (size_t)nc * plan.esz;
    const long long rest = inner[1];
    const bool T = d[0] > 1 && d[1] > 1 && (size_t)d[1] * rest * plan.esz >= (size_t)256 * 1024;
    plan.transposed = false; // the 3-D line maps of W do not apply
    int rc, vz = -1;
    if (!real && nl > 1 && (rc = need_variant(plan, nl, &vz))) return rc;
    if (vz >= 0) vz = contig_variant(plan.prec, nl);
    // one strided pass per axis before the last, standard layout, indexed by axis
    std::vector<Pass> ax(r);
    std::vector<bool> has(r, false);
    for (int i = r - 2; i >= 0; --i) {
        if (d[i] == 1) continue;
        int v;
        if ((rc = need_variant(plan, d[i], &v))) return rc;
        if (inner[i] >= (1LL << 31) || outer[i] >= (1LL << 31))
            return set_error(MIFFT_ERR_UNSUPPORTED, "axis %d: %lld columns x %lld groups is too large", i,
                             inner[i], outer[i]);
        if ((rc = make_strided(plan, ax[i], d[i], (int)inner[i], (int)outer[i], inner[i], d[i] * inner[i], v, 0)))
            return rc;
        ax[i].tag = i == r - 2 ? 1 : 2;
        has[i] = true;
    }
    Pass a1w, a0w; // with W: axis 1 writing W, axis 0 reading it
    if (T) {
        a1w = ax[1];
        a1w.es_out = (long long)d[0] * rest;
        a1w.gs_out = rest;
        if ((rc = make_strided(plan, a0w, d[0], (int)rest, d[1], rest, (long long)d[0] * rest, ax[0].vidx, 0)))
            return rc;
        a0w.es_out = (long long)d[1] * rest;
        a0w.gs_out = rest;
        a0w.tag = 2;
    }
    Pass zf, zi;
    const bool has_z = real || nl > 1;
    if (real) {
        if ((rc = make_real_z(plan, zf, P_R2C, lines)) || (rc = make_real_z(plan, zi, P_C2R, lines))) return rc;
    } else if (has_z) {
        if ((rc = make_contig(plan, zf, nl, lines, vz))) return rc;
        zi = zf;
        zi.sgn = -1;
    }
    zf.tag = zi.tag = 0;
    zf.sgn = +1;
    auto with = [](Pass q, int sgn, BufId src, BufId dst, long long off_in = 0, long long off_out = 0) {
        q.sgn = sgn;
        q.src = src;
        q.dst = dst;
        q.off_in = off_in;
        q.off_out = off_out;
        return q;
    };
    // forward: z, then the strided axes last to first; in -> out, then in place
    auto& f = plan.fwd;
    f.clear();
    if (has_z) f.push_back(with(zf, +1, B_IN, B_OUT));
    for (int i = r - 2; i >= (T ? 2 : 0); --i)
        if (has[i]) f.push_back(with(ax[i], +1, f.empty() ? B_IN : B_OUT, B_OUT));
    if (T) {
        f.push_back(with(a1w, +1, f.empty() ? B_IN : B_OUT, B_WS));
        f.push_back(with(a0w, +1, B_WS, B_OUT));
    }
    // inverse.  C2C: the first pass reads the input, the rest run in place on
    // out.  R2C: the complex passes run in the workspace (after W, in its
    // second spectrum), and the C2R reads it (or the input if it is alone).
    auto& v = plan.inv;
    v.clear();
    const BufId work = real ? B_WS : B_OUT;
    const long long woff = real && T ? (long long)spec_bytes : 0;
    if (T) {
        v.push_back(with(a1w, -1, B_IN, B_WS));
        v.push_back(with(a0w, -1, B_WS, work, 0, woff));
    }
    for (int i = T ? 2 : 0; i <= r - 2; ++i)
        if (has[i]) v.push_back(with(ax[i], -1, v.empty() ? B_IN : work, work, woff, woff));
    if (real)
        v.push_back(with(zi, -1, v.empty() ? B_IN : B_WS, B_OUT, v.empty() ? 0 : woff, 0));
    else if (has_z)
        v.push_back(with(zi, -1, v.empty() ? B_IN : B_OUT, B_OUT));
    for (auto* list : {&plan.fwd, &plan.inv})
        if (list->empty()) { // every extent 1: the identity
            Pass c;
            c.kind = P_COPY;
            c.bytes = plan.esz;
            c.src = B_IN;
            c.dst = B_OUT;
            list->push_back(c);
        }
    bool uses_ws = false;
    for (auto* list : {&plan.fwd, &plan.inv})
        for (const Pass& q : *list) uses_ws |= q.src == B_WS || q.dst == B_WS;
    plan.ws_bytes = !uses_ws ? 0 : (real && T ? 2 * spec_bytes : spec_bytes);
    plan.default_ws_bytes = plan.ws_bytes;
    plan.poisson.clear();
    plan.poisson_ws_bytes = 0;
    tile_passes(plan);
    return validate_extents(plan);
}

} // namespace mifft
