// batch.hip -- host side of the batched uneven-size executor.
//
// mifft_batch_create builds the queue of work items of a batch of 3-D C2C
// transforms (z-passes of every transform, then y-passes, then x-passes; see
// batch_kernels.hpp), uploads the pass table, generates twiddles per distinct
// length and sizes the persistent grid.  Execution is one reset kernel and
// one persistent kernel; mifft_batch_graph_launch captures the two into a
// HIP graph once per set of buffers and replays it.  With MIFFT_BATCH_KERNELS
// the batch runs instead as the per-pass kernels of ordinary plans (one plan
// per distinct shape), which also covers lengths outside the persistent
// kernel's menu.
#include <algorithm>
#include <cstdlib>
#include <cstring>
#include <map>
#include <mutex>
#include <set>
#include <vector>

#include "aux_kernels.hpp"
#include "batch_kernels.hpp"
#include "plan.hpp"

extern "C" {
hipError_t mifft_batch_launch_float(const void*, unsigned, size_t, int*, int, hipStream_t);
hipError_t mifft_batch_launch_double(const void*, unsigned, size_t, int*, int, hipStream_t);
int mifft_batch_blocks_per_cu_float(size_t);
int mifft_batch_blocks_per_cu_double(size_t);
int mifft_plan_create(mifft_plan*, int, int, int, int, int, unsigned);
int mifft_execute_forward(mifft_plan, const void*, void*, void*);
int mifft_plan_destroy(mifft_plan);
}

struct mifft_batch_s {
    int count = 0, prec = MIFFT_FP32;
    bool kernels = false; // per-pass kernel launches instead of the persistent kernel
    bool grouped = false; // kernels: each pass of all transforms of one shape as one launch
    std::vector<int> dims;
    // persistent path
    std::vector<mifft::BatchPass> passes;
    mifft::BatchPass* d_passes = nullptr;
    int* d_item_pass = nullptr; // pass index of every queue item
    int* d_counters = nullptr;
    int ncounters = 0;
    int total_items = 0;
    int stage_items[mifft::kBatchStages] = {0, 0, 0};
    int publish_every = 1 << 30; // completions a workgroup holds at most before publishing
    unsigned grid = 0;
    size_t lds = 0;
    std::map<int, void*> tw;
    int dev = 0;
    // per (stage, line length): code-path variant and queue item size (KiB);
    // the defaults are variant 0 and 64 KiB (MIFFT_BATCH_ITEM_KIB overrides)
    std::map<std::pair<int, int>, std::pair<int, int>> choice;
    // per-pass kernel path: one plan per distinct shape
    std::map<std::vector<int>, mifft_plan> plans;
    // graph replay
    hipStream_t cap_stream = nullptr;
    hipGraph_t graph = nullptr;
    hipGraphExec_t exec = nullptr;
    std::vector<const void*> g_in;
    std::vector<void*> g_out;
    ~mifft_batch_s();
};

namespace mifft {

static std::mutex g_bmu;
static std::set<const void*> g_blive;

static bool batch_live(const void* b)
{
    std::lock_guard<std::mutex> g(g_bmu);
    return g_blive.count(b) != 0;
}

static const int kMenu[] = {
#define MIFFT_BATCH_LEN(I, LEN) LEN,
    MIFFT_BATCH_MENU(MIFFT_BATCH_LEN)
#undef MIFFT_BATCH_LEN
};
static const int kMenuN = (int)(sizeof(kMenu) / sizeof(kMenu[0]));

static int menu_code(int L)
{
    for (int i = 0; i < kMenuN; ++i)
        if (kMenu[i] == L) return i;
    return -1;
}

} // namespace mifft

mifft_batch_s::~mifft_batch_s()
{
    if (exec) hipGraphExecDestroy(exec);
    if (graph) hipGraphDestroy(graph);
    if (cap_stream) hipStreamDestroy(cap_stream);
    if (d_passes) hipFree(d_passes);
    if (d_item_pass) hipFree(d_item_pass);
    if (d_counters) hipFree(d_counters);
    for (auto& kv : tw) hipFree(kv.second);
    for (auto& kv : plans) mifft_plan_destroy(kv.second);
}

namespace mifft {

static int batch_enqueue(mifft_batch b, void* const* in, void* const* out, hipStream_t s);

static void free_tables(mifft_batch_s* b)
{
    if (b->d_passes) hipFree(b->d_passes);
    if (b->d_item_pass) hipFree(b->d_item_pass);
    if (b->d_counters) hipFree(b->d_counters);
    b->d_passes = nullptr;
    b->d_item_pass = nullptr;
    b->d_counters = nullptr;
}

// (Re)build the work queue of the persistent kernel from b->dims and the
// per-(stage, length) choices, upload its tables and size the grid.
static int build_queue(mifft_batch_s* b)
{
    const int count = b->count, prec = b->prec;
    const int* dims = b->dims.data();
    const size_t esz = prec == MIFFT_FP64 ? 16 : 8;
    free_tables(b);
    b->passes.clear();
    for (int k = 0; k < kBatchStages; ++k) b->stage_items[k] = 0;
    // ---- passes in queue order: all z, then all y, then all x
    std::vector<BatchPass>& P = b->passes;
    std::vector<int> last(count, -1); // index of each transform's latest pass
    size_t max_lds = 0; // dynamic LDS elements of the largest pass
    // data per queue item (MIFFT_BATCH_ITEM_KIB overrides the 128 KiB default;
    // untuned 64-transform batch: 64 KiB 1.09 ms, 128 KiB 1.04, 256 KiB 1.03)
    size_t default_item = 128 * 1024;
    if (const char* e = getenv("MIFFT_BATCH_ITEM_KIB")) {
        const long v = atol(e);
        if (v > 0 && v <= 64 * 1024) default_item = (size_t)v * 1024;
    }
    for (int stage = 0; stage < 3; ++stage) {
        // Within a stage the passes are ordered by line length, so that the
        // workgroups running at any moment mostly execute the same
        // per-length code (one instruction-cache working set, not many).
        std::vector<int> order(count);
        for (int t = 0; t < count; ++t) order[t] = t;
        auto len_of = [&](int t) { return dims[3 * t + (stage == 0 ? 2 : (stage == 1 ? 1 : 0))]; };
        std::stable_sort(order.begin(), order.end(), [&](int a, int c) { return len_of(a) < len_of(c); });
        for (int t : order) {
            const int n0 = dims[3 * t], n1 = dims[3 * t + 1], n2 = dims[3 * t + 2];
            const int L = stage == 0 ? n2 : (stage == 1 ? n1 : n0);
            if (L == 1) continue;
            int var = 0;
            size_t item_bytes = default_item;
            auto ch = b->choice.find({stage, L});
            if (ch != b->choice.end()) {
                var = batch_var_distinct(L, ch->second.first) ? ch->second.first : 0;
                item_bytes = (size_t)ch->second.second * 1024;
            }
            BatchPass p{};
            p.kind = stage == 0 ? 0 : 1;
            p.code = kBatchVariants * menu_code(L) + var;
            p.L = L;
            p.tpl = threads_per_line(L, batch_var_policy(var), batch_var_emul(var));
            p.xform = t;
            p.from_in = last[t] < 0 ? 1 : 0;
            // z: lines per wavefront sub-tile; y / x: columns per workgroup tile
            p.per_wave = stage == 0 ? 64 / p.tpl : batch_tile_cols(p.tpl);
            if (stage == 0) {
                p.units = (long long)n0 * n1;
                p.subtiles = (int)((p.units + p.per_wave - 1) / p.per_wave);
            } else if (stage == 1) {
                p.cols = n2;
                p.gs = (long long)n1 * n2;
                p.es = n2;
                p.subtiles_per_group = (p.cols + p.per_wave - 1) / p.per_wave;
                p.subtiles = p.subtiles_per_group * n0;
                p.units = (long long)n0 * n2;
            } else {
                p.cols = n1 * n2;
                p.gs = 0;
                p.es = (long long)n1 * n2;
                p.subtiles_per_group = (p.cols + p.per_wave - 1) / p.per_wave;
                p.subtiles = p.subtiles_per_group;
                p.units = p.cols;
            }
            // queue items of ~item_bytes of data; z items are a multiple of the
            // wavefronts per workgroup (one sub-tile run per wavefront)
            const size_t sub_bytes = (size_t)p.per_wave * L * esz;
            const int unit = stage == 0 ? kBatchWaves : 1;
            int spi = (int)((item_bytes + sub_bytes * unit - 1) / (sub_bytes * unit)) * unit;
            spi = std::max(unit, std::min(spi, ((p.subtiles + unit - 1) / unit) * unit));
            p.sub_per_item = spi;
            p.nitems = (p.subtiles + spi - 1) / spi;
            p.stage = stage;
            p.dep = last[t];
            p.dep_target = last[t] >= 0 ? P[last[t]].nitems : 0;
            p.dep_stage = last[t] >= 0 ? P[last[t]].stage : 0;
            p.done = (int)P.size();
            auto it = b->tw.find(L);
            if (it == b->tw.end()) {
                void* w = nullptr;
                if (hipMalloc(&w, (size_t)L * esz) != hipSuccess) return set_error(MIFFT_ERR_NOMEM, "twiddles");
                hipError_t e = prec == MIFFT_FP64 ? launch_twiddles<double>((cx<double>*)w, L, nullptr)
                                                  : launch_twiddles<float>((cx<float>*)w, L, nullptr);
                if (e != hipSuccess) {
                    hipFree(w);
                    return set_error(MIFFT_ERR_DEVICE, "twiddle kernel: %s", hipGetErrorString(e));
                }
                it = b->tw.emplace(L, w).first;
            }
            p.tw = it->second;
            last[t] = (int)P.size();
            P.push_back(p);
            max_lds = std::max(max_lds, (size_t)batch_lds_elems(L, p.tpl, prec == MIFFT_FP32));
        }
    }
    int start = 0;
    for (BatchPass& p : P) {
        p.item_start = start;
        start += p.nitems;
        b->stage_items[p.stage] += p.nitems;
    }
    b->total_items = start;
    b->ncounters = (int)P.size() + 2 + kBatchStages;
    b->lds = max_lds * esz;
    if (b->lds > 160 * 1024)
        return set_error(MIFFT_ERR_UNSUPPORTED, "the chosen code paths need %zu bytes of LDS per workgroup", b->lds);
    std::vector<int> item_pass((size_t)b->total_items);
    for (size_t k = 0; k < P.size(); ++k)
        for (int it = 0; it < P[k].nitems; ++it) item_pass[(size_t)P[k].item_start + it] = (int)k;
    if (hipMalloc(&b->d_item_pass, sizeof(int) * item_pass.size()) != hipSuccess ||
        hipMemcpy(b->d_item_pass, item_pass.data(), sizeof(int) * item_pass.size(), hipMemcpyHostToDevice) !=
            hipSuccess)
        return set_error(MIFFT_ERR_NOMEM, "batch item table");
    if (hipMalloc(&b->d_passes, sizeof(BatchPass) * P.size()) != hipSuccess ||
        hipMalloc(&b->d_counters, sizeof(int) * b->ncounters) != hipSuccess)
        return set_error(MIFFT_ERR_NOMEM, "batch tables");
    if (hipMemcpy(b->d_passes, P.data(), sizeof(BatchPass) * P.size(), hipMemcpyHostToDevice) != hipSuccess ||
        hipMemset(b->d_counters, 0, sizeof(int) * b->ncounters) != hipSuccess)
        return set_error(MIFFT_ERR_DEVICE, "uploading the batch tables");
    hipDeviceProp_t prop;
    if (hipGetDeviceProperties(&prop, b->dev) != hipSuccess) return set_error(MIFFT_ERR_DEVICE, "device properties");
    const int per_cu = prec == MIFFT_FP64 ? mifft_batch_blocks_per_cu_double(b->lds)
                                          : mifft_batch_blocks_per_cu_float(b->lds);
    long long grid = (long long)prop.multiProcessorCount * per_cu;
    if (grid > b->total_items) grid = b->total_items;
    b->grid = (unsigned)std::max(1LL, grid);
    return MIFFT_OK;
}

static const char* const kStageName[kBatchStages] = {"z", "y", "x"};

// MIFFT_TUNE for the persistent kernel: per (stage, line length) of the
// batch, the code-path variant (radix order, radix groups per thread) and
// the queue item size, chosen by timing the whole batch (one persistent
// launch; 2 untimed + 5 timed on scratch buffers of the batch's shapes) for
// each candidate of one (stage, length) at a time while the others keep
// their current choice, the largest (stage, length) by data first --
// planning by measurement as in the MEASURE planner of Sec. 3.  Choices
// stored in the wisdom table (MIFFT_WISDOM) are applied without timing.
static int tune_batch(mifft_batch_s* b)
{
    const size_t esz = b->prec == MIFFT_FP64 ? 16 : 8;
    hipDeviceProp_t prop;
    if (hipGetDeviceProperties(&prop, b->dev) != hipSuccess) return set_error(MIFFT_ERR_DEVICE, "device properties");
    char arch[16];
    snprintf(arch, sizeof(arch), "%.*s", 6, prop.gcnArchName);
    auto key = [&](int stage, int L) {
        char k[96];
        snprintf(k, sizeof(k), "%s|%s|batch_%s|L=%d", arch, b->prec == MIFFT_FP64 ? "fp64" : "fp32",
                 kStageName[stage], L);
        return std::string(k);
    };
    // (stage, length) groups and their data
    std::map<std::pair<int, int>, double> data;
    for (int t = 0; t < b->count; ++t) {
        const int* d = &b->dims[3 * t];
        const double bytes = (double)d[0] * d[1] * d[2] * esz;
        for (int stage = 0; stage < 3; ++stage) {
            const int L = d[stage == 0 ? 2 : (stage == 1 ? 1 : 0)];
            if (L > 1) data[{stage, L}] += bytes;
        }
    }
    std::vector<std::pair<int, int>> todo;
    for (const auto& kv : data) {
        int pol = 0, emul = 1, kib = 128;
        if (wisdom_batch_get(key(kv.first.first, kv.first.second), &pol, &emul, &kib)) {
            const int var = pol == 2 ? 1 : (emul == 2 ? 2 : 0);
            b->choice[kv.first] = {var, kib};
        } else {
            todo.push_back(kv.first);
        }
    }
    if (todo.empty()) return build_queue(b);
    std::sort(todo.begin(), todo.end(), [&](const auto& a, const auto& c) { return data[a] > data[c]; });

    // scratch inputs and outputs of the batch's shapes
    std::vector<void*> in(b->count, nullptr), out(b->count, nullptr);
    hipStream_t s = nullptr;
    hipEvent_t e0 = nullptr, e1 = nullptr;
    int rc = MIFFT_OK;
    for (int t = 0; t < b->count && rc == MIFFT_OK; ++t) {
        const size_t n = (size_t)b->dims[3 * t] * b->dims[3 * t + 1] * b->dims[3 * t + 2] * esz;
        if (hipMalloc(&in[t], n) != hipSuccess || hipMalloc(&out[t], n) != hipSuccess ||
            hipMemset(in[t], 0, n) != hipSuccess)
            rc = set_error(MIFFT_ERR_NOMEM, "tuning scratch buffers");
    }
    if (rc == MIFFT_OK && (hipStreamCreateWithFlags(&s, hipStreamNonBlocking) != hipSuccess ||
                           hipEventCreate(&e0) != hipSuccess || hipEventCreate(&e1) != hipSuccess))
        rc = set_error(MIFFT_ERR_DEVICE, "tuning stream / events");
    // whole-batch time of the current choices, microseconds (-1: failed;
    // -2: the choices do not fit the LDS of a workgroup, not a candidate)
    auto measure = [&]() -> double {
        if (const int e = build_queue(b)) return e == MIFFT_ERR_UNSUPPORTED ? -2 : -1;
        for (int w = 0; w < 2; ++w)
            if (batch_enqueue(b, in.data(), out.data(), s)) return -1;
        hipEventRecord(e0, s);
        for (int r = 0; r < 5; ++r)
            if (batch_enqueue(b, in.data(), out.data(), s)) return -1;
        hipEventRecord(e1, s);
        if (hipEventSynchronize(e1) != hipSuccess) return -1;
        int flag = 0;
        if (hipMemcpy(&flag, b->d_counters + 1 + b->passes.size(), sizeof(int), hipMemcpyDeviceToHost) !=
                hipSuccess ||
            flag)
            return -1;
        float ms = 0;
        hipEventElapsedTime(&ms, e0, e1);
        return ms * 1e3 / 5;
    };
    std::vector<std::pair<std::string, std::vector<double>>> stored;
    for (const auto& g : todo) {
        if (rc) break;
        const int L = g.second;
        std::pair<int, int> best{0, 128};
        double best_us = 1e30;
        for (int var = 0; var < kBatchVariants; ++var) {
            if (!batch_var_distinct(L, var)) continue;
            for (int kib : {32, 64, 128, 256}) {
                b->choice[g] = {var, kib};
                const double us = measure();
                if (us == -2) continue;
                if (us < 0) {
                    rc = set_error(MIFFT_ERR_DEVICE, "tuning run failed (stage %s, L=%d, variant %d)",
                                   kStageName[g.first], L, var);
                    break;
                }
                if (us < best_us) {
                    best_us = us;
                    best = {var, kib};
                }
            }
            if (rc) break;
        }
        b->choice[g] = best;
        stored.push_back({key(g.first, L), {(double)batch_var_policy(best.first), (double)batch_var_emul(best.first),
                                            (double)best.second, best_us}});
    }
    if (s) hipStreamSynchronize(s);
    if (e0) hipEventDestroy(e0);
    if (e1) hipEventDestroy(e1);
    if (s) hipStreamDestroy(s);
    for (void* p : in)
        if (p) hipFree(p);
    for (void* p : out)
        if (p) hipFree(p);
    if (rc) return rc;
    wisdom_batch_put(stored);
    return build_queue(b);
}

int batch_create(mifft_batch* out, int count, const int* dims, int kind, int prec, unsigned flags)
{
    if (!out || !dims) return set_error(MIFFT_ERR_INVALID, "out / dims is NULL");
    if (count < 1) return set_error(MIFFT_ERR_INVALID, "count must be >= 1");
    if (kind != MIFFT_C2C && kind != MIFFT_R2C) return set_error(MIFFT_ERR_INVALID, "bad kind %d", kind);
    if (prec != MIFFT_FP32 && prec != MIFFT_FP64) return set_error(MIFFT_ERR_INVALID, "bad precision %d", prec);
    if (flags & ~(unsigned)(MIFFT_TUNE | MIFFT_BATCH_KERNELS | MIFFT_BATCH_GROUPED))
        return set_error(MIFFT_ERR_INVALID, "unknown flags 0x%x", flags);
    if ((flags & MIFFT_BATCH_GROUPED) && (flags & MIFFT_BATCH_KERNELS))
        return set_error(MIFFT_ERR_INVALID, "MIFFT_BATCH_GROUPED and MIFFT_BATCH_KERNELS exclude each other");
    if (kind != MIFFT_C2C) return set_error(MIFFT_ERR_UNSUPPORTED, "batches are C2C only");
    if (count > kBatchMax) return set_error(MIFFT_ERR_UNSUPPORTED, "at most %d transforms per batch", kBatchMax);
    const bool grouped = flags & MIFFT_BATCH_GROUPED;
    const bool kernels = (flags & MIFFT_BATCH_KERNELS) || grouped;
    for (int t = 0; t < count; ++t)
        for (int a = 0; a < 3; ++a) {
            const int L = dims[3 * t + a];
            if (L < 1) return set_error(MIFFT_ERR_INVALID, "transform %d: extent %d < 1", t, L);
            if (!supported_length(L))
                return set_error(MIFFT_ERR_UNSUPPORTED, "transform %d: length %d unsupported", t, L);
            if (!kernels && L > 1 && menu_code(L) < 0)
                return set_error(MIFFT_ERR_UNSUPPORTED,
                                 "transform %d: length %d has no persistent code path (2..256, factors "
                                 "2, 3, 5); use MIFFT_BATCH_KERNELS",
                                 t, L);
        }
    for (int t = 0; !kernels && t < count; ++t)
        if (dims[3 * t] == 1 && dims[3 * t + 1] == 1 && dims[3 * t + 2] == 1)
            return set_error(MIFFT_ERR_UNSUPPORTED,
                             "transform %d is 1 x 1 x 1 (no pass to run); use MIFFT_BATCH_KERNELS", t);
    int dev = 0;
    int nd = 0;
    if (hipGetDeviceCount(&nd) != hipSuccess || nd < 1)
        return set_error(MIFFT_ERR_DEVICE, "no HIP device available");
    hipGetDevice(&dev);

    mifft_batch_s* b = new mifft_batch_s();
    b->count = count;
    b->prec = prec;
    b->kernels = kernels;
    b->grouped = grouped;
    b->dims.assign(dims, dims + 3 * count);
    const size_t esz = prec == MIFFT_FP64 ? 16 : 8;

    if (kernels) {
        for (int t = 0; t < count; ++t) {
            std::vector<int> key(dims + 3 * t, dims + 3 * t + 3);
            if (b->plans.count(key)) continue;
            mifft_plan p = nullptr;
            int rc = mifft_plan_create(&p, key[0], key[1], key[2], MIFFT_C2C, prec, flags & MIFFT_TUNE);
            if (rc) {
                delete b;
                return rc;
            }
            b->plans[key] = p;
        }
    } else {
        b->dev = dev;
        if (const char* e = getenv("MIFFT_BATCH_PUBLISH_EVERY")) {
            const int v = atoi(e);
            if (v > 0) b->publish_every = v;
        }
        int rc = (flags & MIFFT_TUNE) ? tune_batch(b) : build_queue(b);
        if (rc) {
            delete b;
            return rc;
        }
    }
    hipError_t e = hipDeviceSynchronize();
    if (e != hipSuccess) {
        delete b;
        return set_error(MIFFT_ERR_DEVICE, "batch set-up: %s", hipGetErrorString(e));
    }
    {
        std::lock_guard<std::mutex> g(g_bmu);
        g_blive.insert(b);
    }
    *out = b;
    return MIFFT_OK;
}

// Grouped: pass k of every shape's plan, for all transforms of that shape,
// before pass k + 1 of any; up to kMaxGroup transforms per launch.  A plan
// with a pass that is not a plain contiguous / strided pass on the caller's
// buffers, or that needs a workspace (which the members would share), runs
// per transform instead.
static bool plan_groupable(const Plan& P)
{
    if (P.ws_bytes != 0) return false;
    for (const Pass& q : P.fwd)
        if ((q.kind != P_CONTIG && q.kind != P_STRIDED) || (q.src != B_IN && q.src != B_OUT) ||
            (q.dst != B_IN && q.dst != B_OUT))
            return false;
    return true;
}

static int enqueue_grouped(mifft_batch b, void* const* in, void* const* out, hipStream_t s)
{
    size_t npass = 0;
    for (const auto& kv : b->plans) npass = std::max(npass, plan_of(kv.second)->fwd.size());
    for (size_t k = 0; k < npass; ++k) {
        for (const auto& kv : b->plans) {
            const Plan* P = plan_of(kv.second);
            if (k >= P->fwd.size()) continue;
            std::vector<int> members;
            for (int t = 0; t < b->count; ++t)
                if (std::equal(kv.first.begin(), kv.first.end(), b->dims.begin() + 3 * t)) members.push_back(t);
            if (!plan_groupable(*P)) {
                for (int t : members)
                    if (k == 0) {
                        int rc = mifft_execute_forward(kv.second, in[t], out[t], s);
                        if (rc) return rc;
                    }
                continue;
            }
            const Pass& q = P->fwd[k];
            for (size_t i = 0; i < members.size();) {
                const int ng = (int)std::min<size_t>(kMaxGroup, members.size() - i);
                const void* src[kMaxGroup];
                void* dst[kMaxGroup];
                for (int j = 0; j < ng; ++j) {
                    const int t = members[i + j];
                    src[j] = (q.src == B_IN ? (const char*)in[t] : (const char*)out[t]) + q.off_in;
                    dst[j] = (q.dst == B_IN ? (char*)in[t] : (char*)out[t]) + q.off_out;
                }
                const hipError_t e = ng > 1 ? launch_pass_group(q, b->prec, ng, src, dst, s)
                                            : launch_pass(q, b->prec, src[0], dst[0], s);
                if (e != hipSuccess) return set_error(MIFFT_ERR_DEVICE, "kernel launch: %s", hipGetErrorString(e));
                i += ng;
            }
        }
    }
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return set_error(MIFFT_ERR_DEVICE, "kernel launch: %s", hipGetErrorString(e));
    return MIFFT_OK;
}

static int batch_enqueue(mifft_batch b, void* const* in, void* const* out, hipStream_t s)
{
    if (b->grouped) return enqueue_grouped(b, in, out, s);
    if (b->kernels) {
        for (int t = 0; t < b->count; ++t) {
            std::vector<int> key(b->dims.begin() + 3 * t, b->dims.begin() + 3 * t + 3);
            int rc = mifft_execute_forward(b->plans[key], in[t], out[t], s);
            if (rc) return rc;
        }
        return MIFFT_OK;
    }
    hipError_t e;
    if (b->prec == MIFFT_FP64) {
        BatchArgs<double> a{};
        a.passes = b->d_passes;
        a.item_pass = b->d_item_pass;
        a.npass = (int)b->passes.size();
        a.total_items = b->total_items;
        a.counters = b->d_counters;
        a.spin_limit = 1u << 22;
        a.publish_every = b->publish_every;
        for (int k = 0; k < kBatchStages; ++k) a.stage_items[k] = b->stage_items[k];
        for (int t = 0; t < b->count; ++t) {
            a.in[t] = (const cx<double>*)in[t];
            a.out[t] = (cx<double>*)out[t];
        }
        e = mifft_batch_launch_double(&a, b->grid, b->lds, b->d_counters, b->ncounters, s);
    } else {
        BatchArgs<float> a{};
        a.passes = b->d_passes;
        a.item_pass = b->d_item_pass;
        a.npass = (int)b->passes.size();
        a.total_items = b->total_items;
        a.counters = b->d_counters;
        a.spin_limit = 1u << 22;
        a.publish_every = b->publish_every;
        for (int k = 0; k < kBatchStages; ++k) a.stage_items[k] = b->stage_items[k];
        for (int t = 0; t < b->count; ++t) {
            a.in[t] = (const cx<float>*)in[t];
            a.out[t] = (cx<float>*)out[t];
        }
        e = mifft_batch_launch_float(&a, b->grid, b->lds, b->d_counters, b->ncounters, s);
    }
    if (e != hipSuccess) return set_error(MIFFT_ERR_DEVICE, "batch launch: %s", hipGetErrorString(e));
    return MIFFT_OK;
}

int batch_execute(mifft_batch b, void* const* in, void* const* out, void* stream, bool graph)
{
    if (!b) return set_error(MIFFT_ERR_INVALID, "batch is NULL");
    if (!batch_live(b)) return set_error(MIFFT_ERR_BADPLAN, "handle is not a live batch");
    if (!in || !out) return set_error(MIFFT_ERR_INVALID, "in / out arrays are NULL");
    for (int t = 0; t < b->count; ++t) {
        if (!in[t] || !out[t]) return set_error(MIFFT_ERR_INVALID, "transform %d: NULL buffer", t);
        if (((uintptr_t)in[t] | (uintptr_t)out[t]) & 15u)
            return set_error(MIFFT_ERR_INVALID, "transform %d: buffers must be 16-byte aligned", t);
    }
    hipStream_t s = (hipStream_t)stream;
    if (!graph) return batch_enqueue(b, in, out, s);
    const bool same = b->exec && std::equal(b->g_in.begin(), b->g_in.end(), in) &&
                      std::equal(b->g_out.begin(), b->g_out.end(), out);
    if (!same) {
        if (b->exec) hipGraphExecDestroy(b->exec);
        if (b->graph) hipGraphDestroy(b->graph);
        b->exec = nullptr;
        b->graph = nullptr;
        if (!b->cap_stream && hipStreamCreateWithFlags(&b->cap_stream, hipStreamNonBlocking) != hipSuccess)
            return set_error(MIFFT_ERR_DEVICE, "capture stream");
        hipError_t e = hipStreamBeginCapture(b->cap_stream, hipStreamCaptureModeThreadLocal);
        if (e != hipSuccess) return set_error(MIFFT_ERR_DEVICE, "begin capture: %s", hipGetErrorString(e));
        int rc = batch_enqueue(b, in, out, b->cap_stream);
        hipGraph_t g = nullptr;
        e = hipStreamEndCapture(b->cap_stream, &g);
        if (rc) {
            if (g) hipGraphDestroy(g);
            return rc;
        }
        if (e != hipSuccess) return set_error(MIFFT_ERR_DEVICE, "end capture: %s", hipGetErrorString(e));
        e = hipGraphInstantiate(&b->exec, g, nullptr, nullptr, 0);
        if (e != hipSuccess) {
            hipGraphDestroy(g);
            return set_error(MIFFT_ERR_DEVICE, "graph instantiate: %s", hipGetErrorString(e));
        }
        b->graph = g;
        b->g_in.assign(in, in + b->count);
        b->g_out.assign(out, out + b->count);
    }
    hipError_t e = hipGraphLaunch(b->exec, s);
    if (e != hipSuccess) return set_error(MIFFT_ERR_DEVICE, "graph launch: %s", hipGetErrorString(e));
    return MIFFT_OK;
}

int batch_destroy(mifft_batch b)
{
    if (!b) return MIFFT_OK;
    {
        std::lock_guard<std::mutex> g(g_bmu);
        if (!g_blive.erase(b)) return set_error(MIFFT_ERR_BADPLAN, "handle is not a live batch");
    }
    delete b;
    return MIFFT_OK;
}

int batch_check(mifft_batch b, int* aborted)
{
    if (!b || !aborted) return set_error(MIFFT_ERR_INVALID, "NULL argument");
    if (!batch_live(b)) return set_error(MIFFT_ERR_BADPLAN, "handle is not a live batch");
    *aborted = 0;
    if (b->kernels) return MIFFT_OK;
    int flag = 0;
    hipError_t e = hipMemcpy(&flag, b->d_counters + 1 + b->passes.size(), sizeof(int), hipMemcpyDeviceToHost);
    if (e != hipSuccess) return set_error(MIFFT_ERR_DEVICE, "reading the abort flag: %s", hipGetErrorString(e));
    *aborted = flag;
    return MIFFT_OK;
}

int batch_describe(mifft_batch b, char* buf, size_t len)
{
    if (!b || !buf || !len) return set_error(MIFFT_ERR_INVALID, "NULL argument");
    if (!batch_live(b)) return set_error(MIFFT_ERR_BADPLAN, "handle is not a live batch");
    std::string s;
    char line[256];
    if (b->kernels) {
        snprintf(line, sizeof(line), "mode=%s transforms=%d shapes=%zu\n", b->grouped ? "grouped" : "kernels",
                 b->count, b->plans.size());
        s += line;
    } else {
        snprintf(line, sizeof(line), "mode=persistent transforms=%d passes=%zu items=%d grid=%u block=%d lds=%zu\n",
                 b->count, b->passes.size(), b->total_items, b->grid, kBatchBlock, b->lds);
        s += line;
        // one line per (stage, length): the code path and item size in use
        std::map<std::pair<int, int>, const BatchPass*> seen;
        for (const BatchPass& p : b->passes) seen.emplace(std::make_pair(p.stage, p.L), &p);
        for (const auto& kv : seen) {
            const BatchPass& p = *kv.second;
            const int var = p.code % kBatchVariants;
            snprintf(line, sizeof(line), "stage=%s L=%d variant=%d policy=%d emul=%d tpl=%d sub_per_item=%d%s\n",
                     kStageName[p.stage], p.L, var, batch_var_policy(var), batch_var_emul(var), p.tpl,
                     p.sub_per_item, b->choice.count(kv.first) ? " chosen" : "");
            s += line;
        }
    }
    snprintf(buf, len, "%s", s.c_str());
    return MIFFT_OK;
}

} // namespace mifft
