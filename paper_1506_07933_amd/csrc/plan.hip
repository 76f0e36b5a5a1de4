// plan.hip -- pass lists and launch geometry of a 3-D transform.
//
// Forward (Algorithm 1, left column, at P0 = P1 = 1): z-pass on the
// contiguous axis, then the y-pass (stride n2c), then the x-pass (stride
// n1 n2c).  Inverse (right column): x-pass, y-pass, z-pass.  The first pass
// reads the caller's input; every later pass works in place on the output
// (or, for C2R, on the workspace, so the input is preserved).
#include <cstdio>
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

void set_contig_geometry(Pass& p, int prec, int tpl, int L, long long nlines, int lds_len)
{
    const size_t esz = prec == MIFFT_FP64 ? 16 : 8;
    int lpw = 256 / tpl;
    if (lpw < 1) lpw = 1;
    while (lpw > 1 && (size_t)lpw * lds_len * esz > kLdsBudget) lpw /= 2;
    // keep enough workgroups to fill the chip when the batch is small
    while (lpw > 1 && (nlines + lpw - 1) / lpw < 1024) lpw /= 2;
    p.L = L;
    p.nlines = nlines;
    p.lines_per_wg = lpw;
    p.grid = (unsigned)((nlines + lpw - 1) / lpw);
    p.block = (unsigned)(lpw * tpl);
    p.shmem = (size_t)lpw * lds_len * esz;
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
    } else {
        while (B * tpl < 256 && B < 64) B *= 2;
        while (B > 1 && ((size_t)B * tpl > 1024 || (size_t)B * L * esz > kLdsBudget)) B /= 2;
        int cp = 1 << ilog2(cols < 1 ? 1 : cols);
        if (cp < B) B = cp;
    }
    p.L = L;
    p.B = B;
    p.log2B = ilog2(B);
    p.cols = cols;
    p.groups = groups;
    p.tiles_per_group = (cols + B - 1) / B;
    p.grid = (unsigned)((long long)p.tiles_per_group * groups);
    p.block = (unsigned)(B * tpl);
    p.shmem = (size_t)B * L * esz;
}

// ----------------------------------------------------------------- launch

template <typename T>
static hipError_t launch_fft(const Pass& p, const void* src, void* dst, hipStream_t s)
{
    const Variant<T>& v = table<T>()[p.vidx];
    using V = cx<T>;
    switch (p.kind) {
    case P_CONTIG:
    case P_CONTIG_PACK: {
        ContigArgs<T> a;
        a.in = (const V*)src;
        a.out = (V*)dst;
        a.tw = (const V*)p.tw;
        a.nlines = (int)p.nlines;
        a.lines_per_wg = p.lines_per_wg;
        a.sgn = (T)p.sgn;
        a.pm = p.fd;
        a.pblk = p.blk;
        auto fn = p.kind == P_CONTIG ? v.contig : v.contig_pack;
        hipLaunchKernelGGL(fn, dim3(p.grid), dim3(p.block), p.shmem, s, a);
        break;
    }
    case P_STRIDED:
    case P_STRIDED_SPLIT: {
        StridedArgs<T> a;
        a.in = (const V*)src;
        a.out = (V*)dst;
        a.tw = (const V*)p.tw;
        a.B = p.B;
        a.log2B = p.log2B;
        a.cols = p.cols;
        a.tiles_per_group = p.tiles_per_group;
        a.gs_in = p.gs_in;
        a.gs_out = p.gs_out;
        a.es_in = p.es_in;
        a.es_out = p.es_out;
        a.sgn = (T)p.sgn;
        a.split = p.fd;
        a.s_hi = p.blk;
        auto fn = p.kind == P_STRIDED ? v.strided : v.strided_split;
        hipLaunchKernelGGL(fn, dim3(p.grid), dim3(p.block), p.shmem, s, a);
        break;
    }
    case P_R2C:
    case P_C2R: {
        RealArgs<T> a;
        a.in = src;
        a.out = dst;
        a.tw = (const V*)p.tw;
        a.tw2 = (const V*)p.tw2;
        a.nlines = (int)p.nlines;
        a.lines_per_wg = p.lines_per_wg;
        auto fn = p.kind == P_R2C ? v.r2c : v.c2r;
        hipLaunchKernelGGL(fn, dim3(p.grid), dim3(p.block), p.shmem, s, a);
        break;
    }
    case P_POISSON:
        return launch_poisson<T>((V*)dst, p.n0, p.n1, p.n2c, (T)p.scale, s);
    case P_PACK:
        return launch_pack<T>((const V*)src, (V*)dst, p.n0, p.n1, p.p1, p.M, s);
    case P_UNPACK:
        return launch_unpack<T>((const V*)src, (V*)dst, p.n0, p.n1, p.p1, p.M, s);
    case P_COPY:
        return launch_copy(src, dst, p.bytes, s);
    }
    return hipGetLastError();
}

hipError_t launch_pass(const Pass& p, int prec, const void* src, void* dst, hipStream_t s)
{
    if (prec == MIFFT_FP64) return launch_fft<double>(p, src, dst, s);
    return launch_fft<float>(p, src, dst, s);
}

// --------------------------------------------------------------- twiddles

int get_twiddles(Plan& plan, int L, void** out)
{
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

static int make_strided(Plan& plan, Pass& p, int L, int cols, int groups, long long es,
                        long long gs, int vidx, int forceB)
{
    p.kind = P_STRIDED;
    p.vidx = vidx;
    int rc = get_twiddles(plan, L, (void**)&p.tw);
    if (rc) return rc;
    set_strided_geometry(p, plan.prec, variant_tpl(plan.prec, vidx), L, cols, groups, forceB);
    p.es_in = p.es_out = es;
    p.gs_in = p.gs_out = gs;
    return MIFFT_OK;
}

// Pass over axis `axis` (0 = x, 1 = y, 2 = z) of a complex [n0][n1][nc] array.
static int make_axis_pass(Plan& plan, Pass& p, int axis, int nc, int sgn)
{
    const int n[3] = {plan.n0, plan.n1, nc};
    const int L = n[axis];
    const int vidx = default_variant(plan.prec, L);
    if (vidx < 0) return set_error(MIFFT_ERR_UNSUPPORTED, "no kernel for length %d", L);
    int rc;
    if (axis == 2)
        rc = make_contig(plan, p, L, (long long)plan.n0 * plan.n1, vidx);
    else if (axis == 1)
        rc = make_strided(plan, p, L, nc, plan.n0, nc, (long long)plan.n1 * nc, vidx, 0);
    else
        rc = make_strided(plan, p, L, plan.n1 * nc, 1, (long long)plan.n1 * nc, 0, vidx, 0);
    p.sgn = sgn;
    return rc;
}

static int make_real_z(Plan& plan, Pass& p, PassKind kind)
{
    const int M = plan.n2 / 2;
    const int vidx = default_variant(plan.prec, M);
    if (vidx < 0) return set_error(MIFFT_ERR_UNSUPPORTED, "no kernel for half length %d", M);
    p.kind = kind;
    p.vidx = vidx;
    int rc = get_twiddles(plan, M, (void**)&p.tw);
    if (rc) return rc;
    rc = get_twiddles(plan, plan.n2, (void**)&p.tw2);
    if (rc) return rc;
    set_contig_geometry(p, plan.prec, variant_tpl(plan.prec, vidx), M,
                        (long long)plan.n0 * plan.n1, lds_padded_len(M + 1));
    return MIFFT_OK;
}

int build_plan(Plan& plan, unsigned /*flags*/)
{
    const bool real = plan.kind == MIFFT_R2C;
    const int nc = real ? plan.n2 / 2 + 1 : plan.n2;
    const size_t half_bytes = (size_t)plan.n0 * plan.n1 * nc * plan.esz;
    int rc;
    // ---- forward: z, y, x
    if (real) {
        Pass z;
        if ((rc = make_real_z(plan, z, P_R2C))) return rc;
        z.src = B_IN;
        z.dst = B_OUT;
        plan.fwd.push_back(z);
    } else if (plan.n2 > 1) {
        Pass z;
        if ((rc = make_axis_pass(plan, z, 2, nc, +1))) return rc;
        plan.fwd.push_back(z);
    }
    if (plan.n1 > 1) {
        Pass y;
        if ((rc = make_axis_pass(plan, y, 1, nc, +1))) return rc;
        plan.fwd.push_back(y);
    }
    if (plan.n0 > 1) {
        Pass x;
        if ((rc = make_axis_pass(plan, x, 0, nc, +1))) return rc;
        plan.fwd.push_back(x);
    }
    // ---- inverse: x, y, z
    if (plan.n0 > 1) {
        Pass x;
        if ((rc = make_axis_pass(plan, x, 0, nc, -1))) return rc;
        plan.inv.push_back(x);
    }
    if (plan.n1 > 1) {
        Pass y;
        if ((rc = make_axis_pass(plan, y, 1, nc, -1))) return rc;
        plan.inv.push_back(y);
    }
    if (real) {
        Pass z;
        if ((rc = make_real_z(plan, z, P_C2R))) return rc;
        plan.inv.push_back(z);
    } else if (plan.n2 > 1) {
        Pass z;
        if ((rc = make_axis_pass(plan, z, 2, nc, -1))) return rc;
        plan.inv.push_back(z);
    }
    // ---- buffers: the first pass reads the input, the others run in place
    if (!real) {
        for (auto* list : {&plan.fwd, &plan.inv}) {
            for (size_t i = 0; i < list->size(); ++i) {
                (*list)[i].src = i == 0 ? B_IN : B_OUT;
                (*list)[i].dst = B_OUT;
            }
            if (list->empty()) { // 1 x 1 x 1: the transform is the identity
                Pass c;
                c.kind = P_COPY;
                c.bytes = plan.esz;
                c.src = B_IN;
                c.dst = B_OUT;
                list->push_back(c);
            }
        }
    } else {
        for (size_t i = 1; i < plan.fwd.size(); ++i) plan.fwd[i].src = plan.fwd[i].dst = B_OUT;
        // C2R: complex passes go input -> workspace -> workspace, the last
        // (z) pass reads the workspace (or the input if it is the only pass).
        for (size_t i = 0; i + 1 < plan.inv.size(); ++i) {
            plan.inv[i].src = i == 0 ? B_IN : B_WS;
            plan.inv[i].dst = B_WS;
        }
        plan.inv.back().src = plan.inv.size() == 1 ? B_IN : B_WS;
        plan.inv.back().dst = B_OUT;
        plan.ws_bytes = plan.inv.size() > 1 ? half_bytes : 0;
        // Poisson: R2C into the workspace, y, x, multiply, x^-1, y^-1, C2R out.
        plan.poisson.clear();
        Pass z = plan.fwd[0];
        z.src = B_IN;
        z.dst = B_WS;
        plan.poisson.push_back(z);
        for (size_t i = 1; i < plan.fwd.size(); ++i) {
            Pass q = plan.fwd[i];
            q.src = q.dst = B_WS;
            plan.poisson.push_back(q);
        }
        Pass m;
        m.kind = P_POISSON;
        m.n0 = plan.n0;
        m.n1 = plan.n1;
        m.n2c = nc;
        m.scale = 1.0 / ((double)plan.n0 * plan.n1 * plan.n2);
        m.src = m.dst = B_WS;
        plan.poisson.push_back(m);
        for (size_t i = 0; i < plan.inv.size(); ++i) {
            Pass q = plan.inv[i];
            q.src = B_WS;
            q.dst = (i + 1 == plan.inv.size()) ? B_OUT : B_WS;
            plan.poisson.push_back(q);
        }
        plan.poisson_ws_bytes = half_bytes;
        if (plan.poisson_ws_bytes > plan.ws_bytes) plan.ws_bytes = plan.poisson_ws_bytes;
    }
    return MIFFT_OK;
}

int build_pencil(Plan& plan, unsigned /*flags*/)
{
    const int n0l = plan.n0 / plan.p0, n1l = plan.n1 / plan.p1, N1 = plan.n1, N2 = plan.n2;
    const int M = N2 / plan.p1;
    const long long lines = (long long)n0l * n1l;
    int rc;
    const int vz = default_variant(plan.prec, N2);
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
    return MIFFT_OK;
}

} // namespace mifft
