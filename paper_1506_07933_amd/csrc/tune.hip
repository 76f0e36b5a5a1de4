// tune.hip -- MIFFT_TUNE: measure the compiled alternatives of every pass of a
// plan and keep the fastest (planning by measurement, in the spirit of the
// MEASURE planner the paper builds its libraries with, Sec. 3).
//
// For a contiguous or real pass the candidates are every compiled variant of
// its line length (radix order, elements per thread) times the lines per
// workgroup; for a strided pass, every variant times the column-tile width B.
// Each candidate runs on scratch buffers of the plan's size, 2 untimed + 5
// timed launches on a private stream, and the minimum time wins.  Choices are
// kept in a process-wide wisdom table keyed by device architecture,
// precision, pass kind and geometry; when MIFFT_WISDOM names a file the table
// is loaded from it once and written back (atomically) after every tuning,
// so a restarted process reuses tuned plans without timing them again.
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <fstream>
#include <map>
#include <mutex>
#include <sstream>
#include <string>
#include <vector>

#include "plan.hpp"

namespace mifft {

struct Choice {
    int policy, emul, B, lpw;
    double us;
};

static std::mutex g_wmu;
static std::map<std::string, Choice> g_wisdom;
static bool g_wisdom_loaded = false;

static const char* wisdom_path() { return getenv("MIFFT_WISDOM"); }

// A strided kernel maps thread tid to column tid & (B - 1) and line thread
// tid >> log2(B), which covers each column once only for B a power of two;
// tiles are at most 64 columns wide and 1024 threads.  A contiguous pass
// takes 1 .. 32 lines per workgroup.  Entries of a wisdom file (which may
// have been edited by hand) outside these ranges are ignored.
static bool pow2_in(int v, int lo, int hi) { return v >= lo && v <= hi && (v & (v - 1)) == 0; }
static bool choice_shape_ok(const Choice& c)
{
    if (c.policy < 0 || c.policy > 2 || c.emul < 1 || c.emul > 2) return false;
    return (c.B == 0 && c.lpw >= 1 && c.lpw <= 32) || (c.lpw == 0 && pow2_in(c.B, 1, 64));
}

// Entries of the batched executor ("...|batch_z|L=..", "..._y", "..._x"):
// policy 0 or 2, one or two radix groups per thread, B = the queue item
// size in KiB (32, 64, 128 or 256), lpw unused (0).
static bool is_batch_key(const std::string& k) { return k.find("|batch_") != std::string::npos; }
static bool batch_choice_ok(const Choice& c)
{
    return (c.policy == 0 || c.policy == 2) && (c.emul == 1 || c.emul == 2) &&
           (c.B == 32 || c.B == 64 || c.B == 128 || c.B == 256) && c.lpw == 0;
}

// One entry per line:  "key": [policy, emul, B, lpw, microseconds],
static void load_wisdom_locked()
{
    if (g_wisdom_loaded) return;
    g_wisdom_loaded = true;
    const char* path = wisdom_path();
    if (!path) return;
    std::ifstream f(path);
    std::string line;
    while (std::getline(f, line)) {
        const size_t a = line.find('"'), b = line.find('"', a + 1), c = line.find('[', b);
        if (a == std::string::npos || b == std::string::npos || c == std::string::npos) continue;
        Choice ch;
        const std::string key = line.substr(a + 1, b - a - 1);
        if (sscanf(line.c_str() + c, "[%d, %d, %d, %d, %lf]", &ch.policy, &ch.emul, &ch.B, &ch.lpw, &ch.us) == 5 &&
            (is_batch_key(key) ? batch_choice_ok(ch) : choice_shape_ok(ch)))
            g_wisdom[key] = ch;
    }
}

static void save_wisdom_locked()
{
    const char* path = wisdom_path();
    if (!path) return;
    std::string tmp = std::string(path) + ".tmp";
    {
        std::ofstream f(tmp);
        f << "{\n";
        size_t i = 0;
        for (const auto& kv : g_wisdom) {
            char buf[128];
            snprintf(buf, sizeof(buf), "[%d, %d, %d, %d, %.3f]", kv.second.policy, kv.second.emul, kv.second.B,
                     kv.second.lpw, kv.second.us);
            f << "  \"" << kv.first << "\": " << buf << (++i < g_wisdom.size() ? ",\n" : "\n");
        }
        f << "}\n";
    }
    std::rename(tmp.c_str(), path);
}

static std::string pass_key(const Plan& plan, const Pass& p, const char* arch)
{
    static const char* kn[] = {"contig", "contig_pack", "strided", "strided_unpack", "r2c_z",    "c2r_z",
                               "poisson", "pack",       "unpack",  "copy",           "poisson_x", "strided_pack"};
    std::ostringstream k;
    k << arch << "|" << (plan.prec == MIFFT_FP64 ? "fp64" : "fp32") << "|" << kn[p.kind] << "|L=" << p.L;
    if (p.kind == P_STRIDED || p.kind == P_STRIDED_SPLIT) {
        k << "|cols=" << p.cols << "|groups=" << p.groups << "|es=" << p.es_in << "/" << p.es_out
          << "|gs=" << p.gs_in << "/" << p.gs_out;
        if (p.gdiv_in > 1 || p.gdiv_out > 1)
            k << "|gdiv=" << p.gdiv_in << "/" << p.gdiv_out << "|gs2=" << p.gs2_in << "/" << p.gs2_out;
    }
    else
        k << "|lines=" << p.nlines;
    return k.str();
}

static bool is_tunable(const Pass& p)
{
    return p.kind == P_CONTIG || p.kind == P_STRIDED || p.kind == P_R2C || p.kind == P_C2R;
}

static int lds_len_of(const Pass& p)
{
    return (p.kind == P_R2C || p.kind == P_C2R) ? lds_padded_len(p.L + 1) : lds_padded_len(p.L);
}

// Re-shape pass p for (variant, B or lpw), keeping its buffers and strides.
static bool apply_choice(const Plan& plan, Pass& p, int vidx, int shape)
{
    const int tpl = variant_tpl(plan.prec, vidx);
    const size_t esz = plan.esz;
    if (p.kind == P_STRIDED) {
        const int B = shape;
        if (!pow2_in(B, 1, 64) || (long long)B * tpl > 1024 || (size_t)(B + 1) * p.L * esz > 160 * 1024)
            return false;
        if (p.fixedB && B != p.fixedB) return false; // the tile width is part of a blocked layout
        int lg = 0;
        while ((1 << lg) < B) ++lg;
        p.vidx = vidx;
        p.B = B;
        p.log2B = lg;
        p.block = (unsigned)(B * tpl);
        p.shmem = ((size_t)B * p.L + p.L) * esz;
        tile_pass(plan, p);
        return true;
    }
    const int lpw = shape;
    if (lpw < 1 || lpw > 32 || (long long)lpw * tpl > 1024 || ((size_t)lpw * lds_len_of(p) + p.L) * esz > 160 * 1024)
        return false;
    const int ni = p.ni;
    const long long is_o = p.is_o, is_i = p.is_i, os_o = p.os_o, os_i = p.os_i;
    p.vidx = vidx;
    p.lines_per_wg = lpw;
    p.grid = (unsigned)((p.nlines + lpw - 1) / lpw);
    p.block = (unsigned)(lpw * tpl);
    p.shmem = ((size_t)lpw * lds_len_of(p) + p.L) * esz;
    set_line_map(p, ni, is_o, is_i, os_o, os_i);
    return true;
}

static std::vector<std::pair<int, int>> candidates(const Plan& plan, const Pass& p)
{
    std::vector<std::pair<int, int>> out;
    const int Lv = (p.kind == P_R2C || p.kind == P_C2R) ? p.L : p.L;
    for (int v = 0; v < variant_count(plan.prec); ++v) {
        if (variant_L(plan.prec, v) != Lv) continue;
        const int tpl = variant_tpl(plan.prec, v);
        if (p.kind == P_STRIDED && p.fixedB) {
            out.push_back({v, p.fixedB});
        } else if (p.kind == P_STRIDED) {
            for (int B : {4, 8, 16, 32, 64})
                if ((long long)B * tpl >= 64 || B == 64) out.push_back({v, B});
        } else {
            for (int lpw : {1, 2, 4, 8, 16, 32})
                if ((long long)lpw * tpl >= 64 || lpw == 32) out.push_back({v, lpw});
        }
    }
    return out;
}

// Re-shape every tunable pass that has a wisdom entry; returns whether all had one.
static bool apply_wisdom_locked(Plan& plan, const char* arch)
{
    bool all = true;
    for (auto* list : {&plan.fwd, &plan.inv, &plan.fwd_ip, &plan.inv_ip})
        for (Pass& p : *list) {
            if (!is_tunable(p)) continue;
            auto it = g_wisdom.find(pass_key(plan, p, arch));
            bool done = false;
            if (it != g_wisdom.end()) {
                const int v = find_variant(plan.prec, p.L, it->second.policy, it->second.emul);
                Pass q = p;
                if (v >= 0 && apply_choice(plan, q, v, p.kind == P_STRIDED ? it->second.B : it->second.lpw)) {
                    p = q;
                    done = true;
                }
            }
            all = all && done;
        }
    return all;
}

// Batched executor's choices in the same table (the batch tuner lives in
// batch.hip): look one up, or store several and write the file back.
bool wisdom_batch_get(const std::string& key, int* policy, int* emul, int* item_kib)
{
    std::lock_guard<std::mutex> g(g_wmu);
    load_wisdom_locked();
    auto it = g_wisdom.find(key);
    if (it == g_wisdom.end() || !batch_choice_ok(it->second)) return false;
    *policy = it->second.policy;
    *emul = it->second.emul;
    *item_kib = it->second.B;
    return true;
}

void wisdom_batch_put(const std::vector<std::pair<std::string, std::vector<double>>>& entries)
{
    std::lock_guard<std::mutex> g(g_wmu);
    load_wisdom_locked();
    for (const auto& e : entries) {
        const Choice c{(int)e.second[0], (int)e.second[1], (int)e.second[2], 0, e.second[3]};
        if (batch_choice_ok(c)) g_wisdom[e.first] = c;
    }
    if (!entries.empty()) save_wisdom_locked();
}

int tune_plan(Plan& plan)
{
    char arch[64];
    if (plan.plan_only) {
        // no device: apply the stored choices for the one target this library is built for
        snprintf(arch, sizeof(arch), "gfx950");
        std::lock_guard<std::mutex> g(g_wmu);
        load_wisdom_locked();
        apply_wisdom_locked(plan, arch);
        rebuild_poisson(plan);
        tile_passes(plan);
        return validate_extents(plan);
    }
    hipDeviceProp_t prop;
    if (hipGetDeviceProperties(&prop, plan.device) != hipSuccess)
        return set_error(MIFFT_ERR_DEVICE, "tuning: device properties");
    snprintf(arch, sizeof(arch), "%.*s", 6, prop.gcnArchName);
    std::lock_guard<std::mutex> g(g_wmu);
    load_wisdom_locked();

    const size_t nc = plan.kind == MIFFT_R2C ? plan.n2 / 2 + 1 : plan.n2;
    const size_t cbytes = (size_t)plan.n0 * plan.n1 * nc * plan.esz;
    const size_t rbytes = (size_t)plan.n0 * plan.n1 * plan.n2 * plan.esz / 2;
    // scratch stand-ins for the caller's arrays and for the workspace (whose
    // rows may be padded: it can be larger than the arrays)
    const size_t bytes = std::max(cbytes, rbytes) + 256;
    const size_t wbytes = std::max(bytes, plan.ws_bytes + 256);
    void *A = nullptr, *B = nullptr, *W = nullptr;
    hipStream_t s = nullptr;
    hipEvent_t e0 = nullptr, e1 = nullptr;
    int rc = MIFFT_OK;
    bool tuned_any = false;
    if (hipMalloc(&A, bytes) != hipSuccess || hipMalloc(&B, bytes) != hipSuccess ||
        hipMalloc(&W, wbytes) != hipSuccess || hipStreamCreateWithFlags(&s, hipStreamNonBlocking) != hipSuccess ||
        hipEventCreate(&e0) != hipSuccess || hipEventCreate(&e1) != hipSuccess) {
        rc = set_error(MIFFT_ERR_NOMEM, "tuning scratch buffers");
    } else {
        hipMemsetAsync(A, 0, bytes, s);
        hipMemsetAsync(B, 0, bytes, s);
        hipMemsetAsync(W, 0, wbytes, s);
        auto buf = [&](BufId b) -> void* { return b == B_IN ? A : b == B_WS ? W : B; };
        // a candidate is launched only if its reads and writes stay inside the scratch
        auto fits = [&](const Pass& q) {
            const Extent e = pass_extent(q, plan.esz);
            auto cap = [&](BufId b) { return (long long)((b == B_WS ? wbytes : bytes) / plan.esz); };
            return e.in <= cap(q.src) && e.out <= cap(q.dst);
        };
        for (auto* list : {&plan.fwd, &plan.inv, &plan.fwd_ip, &plan.inv_ip}) {
            for (Pass& p : *list) {
                if (!is_tunable(p)) continue;
                const std::string key = pass_key(plan, p, arch);
                auto it = g_wisdom.find(key);
                if (it != g_wisdom.end()) {
                    const int v = find_variant(plan.prec, p.L, it->second.policy, it->second.emul);
                    if (v >= 0 && apply_choice(plan, p, v, p.kind == P_STRIDED ? it->second.B : it->second.lpw))
                        continue;
                }
                Choice best{-1, -1, 0, 0, 1e30};
                Pass best_pass = p;
                for (auto [v, shape] : candidates(plan, p)) {
                    Pass q = p;
                    if (!apply_choice(plan, q, v, shape) || !fits(q)) continue;
                    bool ok = true;
                    for (int w = 0; w < 2 && ok; ++w)
                        ok = launch_pass(q, plan.prec, buf(q.src), buf(q.dst), s) == hipSuccess;
                    hipEventRecord(e0, s);
                    for (int r = 0; r < 5 && ok; ++r)
                        ok = launch_pass(q, plan.prec, buf(q.src), buf(q.dst), s) == hipSuccess;
                    hipEventRecord(e1, s);
                    if (!ok || hipEventSynchronize(e1) != hipSuccess) {
                        (void)hipGetLastError();
                        continue;
                    }
                    float ms = 0;
                    hipEventElapsedTime(&ms, e0, e1);
                    const double us = ms * 1e3 / 5;
                    if (us < best.us) {
                        best = Choice{variant_policy(plan.prec, v), variant_emul(plan.prec, v),
                                      q.kind == P_STRIDED ? q.B : 0, q.kind == P_STRIDED ? 0 : q.lines_per_wg, us};
                        best_pass = q;
                    }
                }
                if (best.policy >= 0) {
                    p = best_pass;
                    g_wisdom[key] = best;
                    tuned_any = true;
                }
            }
        }
        if (hipStreamSynchronize(s) != hipSuccess) rc = set_error(MIFFT_ERR_DEVICE, "tuning run failed");
    }
    if (e0) hipEventDestroy(e0);
    if (e1) hipEventDestroy(e1);
    if (s) hipStreamDestroy(s);
    if (A) hipFree(A);
    if (B) hipFree(B);
    if (W) hipFree(W);
    if (tuned_any) save_wisdom_locked();
    if (rc == MIFFT_OK) rebuild_poisson(plan);
    if (rc == MIFFT_OK) tile_passes(plan);
    if (rc == MIFFT_OK) rc = validate_extents(plan);
    return rc;
}

} // namespace mifft
