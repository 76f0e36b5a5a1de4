// capi.hip -- the extern "C" entry points declared in include/mifft.h.
//
// Every argument is checked on the host before the first HIP call, so the
// argument errors are the same with or without a device.  Handles are kept
// in a registry so a destroyed or foreign handle is reported as BADPLAN
// instead of being dereferenced.
#include <algorithm>
#include <cstdint>
#include <cstring>
#include <mutex>
#include <set>
#include <string>

#include "aux_kernels.hpp"
#include "plan.hpp"
#include "spectral.hpp"

namespace mifft {
const char* last_error_cstr();
int batch_create(mifft_batch* out, int count, const int* dims, int kind, int prec, unsigned flags);
int batch_execute(mifft_batch b, void* const* in, void* const* out, void* stream, bool graph);
int batch_destroy(mifft_batch b);
int batch_check(mifft_batch b, int* aborted);
int batch_describe(mifft_batch b, char* buf, size_t len);
int tune_plan(Plan& plan);
} // namespace mifft

using namespace mifft;

struct mifft_plan_s : public Plan {};

static_assert(MIFFT_OP_POISSON == OP_POISSON && MIFFT_OP_LAPLACIAN == OP_LAPLACIAN &&
                  MIFFT_OP_HELMHOLTZ == OP_HELMHOLTZ && MIFFT_OP_DX == OP_DX && MIFFT_OP_DY == OP_DY &&
                  MIFFT_OP_DZ == OP_DZ,
              "operator codes of the C ABI and the kernels differ");

static std::mutex g_live_mu;
static std::set<const void*> g_live;

static bool is_live(const void* p)
{
    std::lock_guard<std::mutex> g(g_live_mu);
    return g_live.count(p) != 0;
}

static bool aligned16(const void* p) { return ((uintptr_t)p & 15u) == 0; }

namespace mifft {
const Plan* plan_of(mifft_plan h) { return static_cast<const Plan*>(h); }
} // namespace mifft

static int check_device(int* dev)
{
    int n = 0;
    hipError_t e = hipGetDeviceCount(&n);
    if (e != hipSuccess || n < 1)
        return set_error(MIFFT_ERR_DEVICE, "no HIP device available (%s)",
                         e != hipSuccess ? hipGetErrorString(e) : "0 devices");
    e = hipGetDevice(dev);
    if (e != hipSuccess) return set_error(MIFFT_ERR_DEVICE, "hipGetDevice: %s", hipGetErrorString(e));
    hipDeviceProp_t prop;
    e = hipGetDeviceProperties(&prop, *dev);
    if (e != hipSuccess)
        return set_error(MIFFT_ERR_DEVICE, "hipGetDeviceProperties: %s", hipGetErrorString(e));
    if (strncmp(prop.gcnArchName, "gfx950", 6) != 0)
        return set_error(MIFFT_ERR_DEVICE, "device %d is %s; this library is built for gfx950", *dev,
                         prop.gcnArchName);
    return MIFFT_OK;
}

static int validate_dims(int n0, int n1, int n2, int kind, int prec)
{
    if (kind != MIFFT_C2C && kind != MIFFT_R2C)
        return set_error(MIFFT_ERR_INVALID, "kind %d is not MIFFT_C2C or MIFFT_R2C", kind);
    if (prec != MIFFT_FP32 && prec != MIFFT_FP64)
        return set_error(MIFFT_ERR_INVALID, "precision %d is not MIFFT_FP32 or MIFFT_FP64", prec);
    const int n[3] = {n0, n1, n2};
    for (int i = 0; i < 3; ++i)
        if (n[i] < 1) return set_error(MIFFT_ERR_INVALID, "n%d = %d must be >= 1", i, n[i]);
    for (int i = 0; i < 3; ++i)
        if (!supported_length(n[i]))
            return set_error(MIFFT_ERR_UNSUPPORTED,
                             "n%d = %d: axis lengths must be <= 1024 with prime factors 2, 3, 5", i,
                             n[i]);
    if (kind == MIFFT_R2C && (n2 % 2 != 0))
        return set_error(MIFFT_ERR_UNSUPPORTED, "R2C needs an even n2 (got %d)", n2);
    return MIFFT_OK;
}

static int finish_plan(Plan* p, mifft_plan* out)
{
    hipError_t e = hipStreamSynchronize(nullptr);
    if (e != hipSuccess) {
        delete p;
        return set_error(MIFFT_ERR_DEVICE, "plan set-up: %s", hipGetErrorString(e));
    }
    {
        std::lock_guard<std::mutex> g(g_live_mu);
        g_live.insert(p);
    }
    *out = static_cast<mifft_plan>(p);
    return MIFFT_OK;
}

extern "C" {

static int create_lanes(Plan& p);

int mifft_plan_create(mifft_plan* out, int n0, int n1, int n2, int kind, int prec, unsigned flags)
{
    clear_error();
    if (!out) return set_error(MIFFT_ERR_INVALID, "out is NULL");
    int rc = validate_dims(n0, n1, n2, kind, prec);
    if (rc) return rc;
    if (flags & ~(unsigned)(MIFFT_TUNE | MIFFT_PLAN_ONLY))
        return set_error(MIFFT_ERR_INVALID, "unknown flags 0x%x", flags);
    const bool plan_only = flags & MIFFT_PLAN_ONLY;
    int dev = 0;
    if (!plan_only && (rc = check_device(&dev))) return rc;
    mifft_plan_s* p = new mifft_plan_s();
    p->plan_only = plan_only;
    p->n0 = n0;
    p->n1 = n1;
    p->n2 = n2;
    p->kind = kind;
    p->prec = prec;
    p->device = dev;
    if (!plan_only) {
        int cus = 0;
        if (hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) == hipSuccess && cus > 0)
            p->cus = cus;
    }
    p->esz = prec == MIFFT_FP64 ? 16 : 8;
    if ((rc = build_plan(*p, flags))) {
        delete p;
        return rc;
    }
    if ((flags & MIFFT_TUNE) && (rc = tune_plan(*p))) {
        delete p;
        return rc;
    }
    if (plan_only) {
        std::lock_guard<std::mutex> g(g_live_mu);
        g_live.insert(p);
        *out = static_cast<mifft_plan>(p);
        return MIFFT_OK;
    }
    if (p->default_ws_bytes) {
        hipError_t e = hipMalloc(&p->ws, p->default_ws_bytes);
        if (e != hipSuccess) {
            delete p;
            return set_error(MIFFT_ERR_NOMEM, "workspace of %zu bytes: %s", p->default_ws_bytes,
                             hipGetErrorString(e));
        }
    }
    if ((rc = create_lanes(*p))) {
        delete p;
        return rc;
    }
    return finish_plan(p, out);
}

int mifft_plan_create_nd(mifft_plan* out, int rank, const int* dims, int kind, int prec, unsigned flags)
{
    clear_error();
    if (!out) return set_error(MIFFT_ERR_INVALID, "out is NULL");
    if (!dims) return set_error(MIFFT_ERR_INVALID, "dims is NULL");
    if (rank < 1 || rank > MIFFT_MAX_RANK)
        return set_error(MIFFT_ERR_INVALID, "rank %d must be 1 .. %d", rank, MIFFT_MAX_RANK);
    if (rank <= 3) { // leading extents of 1: the 3-D plan
        int n[3] = {1, 1, 1};
        for (int i = 0; i < rank; ++i) n[3 - rank + i] = dims[i];
        return mifft_plan_create(out, n[0], n[1], n[2], kind, prec, flags);
    }
    if (kind != MIFFT_C2C && kind != MIFFT_R2C)
        return set_error(MIFFT_ERR_INVALID, "kind %d is not MIFFT_C2C or MIFFT_R2C", kind);
    if (prec != MIFFT_FP32 && prec != MIFFT_FP64)
        return set_error(MIFFT_ERR_INVALID, "precision %d is not MIFFT_FP32 or MIFFT_FP64", prec);
    long long total = 1;
    for (int i = 0; i < rank; ++i) {
        if (dims[i] < 1) return set_error(MIFFT_ERR_INVALID, "dims[%d] = %d must be >= 1", i, dims[i]);
        total *= dims[i];
        if (total >= (1LL << 31))
            return set_error(MIFFT_ERR_UNSUPPORTED, "more than 2^31 - 1 elements");
    }
    for (int i = 0; i < rank; ++i)
        if (!supported_length(dims[i]))
            return set_error(MIFFT_ERR_UNSUPPORTED,
                             "dims[%d] = %d: axis lengths must be <= 1024 with prime factors 2, 3, 5", i, dims[i]);
    if (kind == MIFFT_R2C && dims[rank - 1] % 2)
        return set_error(MIFFT_ERR_UNSUPPORTED, "R2C needs an even last extent (got %d)", dims[rank - 1]);
    if (flags & ~(unsigned)(MIFFT_TUNE | MIFFT_PLAN_ONLY))
        return set_error(MIFFT_ERR_INVALID, "unknown flags 0x%x", flags);
    if (flags & MIFFT_TUNE) return set_error(MIFFT_ERR_UNSUPPORTED, "MIFFT_TUNE is offered for rank <= 3");
    int dev = 0, rc;
    const bool plan_only = flags & MIFFT_PLAN_ONLY;
    if (!plan_only && (rc = check_device(&dev))) return rc;
    mifft_plan_s* p = new mifft_plan_s();
    p->plan_only = plan_only;
    p->nd = true;
    p->dims.assign(dims, dims + rank);
    p->n0 = 1;
    for (int i = 0; i + 2 < rank; ++i) p->n0 *= dims[i];
    p->n1 = dims[rank - 2];
    p->n2 = dims[rank - 1];
    p->kind = kind;
    p->prec = prec;
    p->device = dev;
    if (!plan_only) {
        int cus = 0;
        if (hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) == hipSuccess && cus > 0)
            p->cus = cus;
    }
    p->esz = prec == MIFFT_FP64 ? 16 : 8;
    if ((rc = build_nd(*p, flags))) {
        delete p;
        return rc;
    }
    if (plan_only) {
        std::lock_guard<std::mutex> g(g_live_mu);
        g_live.insert(p);
        *out = static_cast<mifft_plan>(p);
        return MIFFT_OK;
    }
    if (p->default_ws_bytes) {
        hipError_t e = hipMalloc(&p->ws, p->default_ws_bytes);
        if (e != hipSuccess) {
            delete p;
            return set_error(MIFFT_ERR_NOMEM, "workspace of %zu bytes: %s", p->default_ws_bytes,
                             hipGetErrorString(e));
        }
    }
    return finish_plan(p, out);
}

int mifft_plan_create_pencil(mifft_plan* out, int n0, int n1, int n2, int p0, int p1, int kind,
                             int prec, unsigned flags)
{
    clear_error();
    if (!out) return set_error(MIFFT_ERR_INVALID, "out is NULL");
    if (kind != MIFFT_C2C && kind != MIFFT_R2C) return set_error(MIFFT_ERR_INVALID, "bad kind %d", kind);
    if (prec != MIFFT_FP32 && prec != MIFFT_FP64)
        return set_error(MIFFT_ERR_INVALID, "bad precision %d", prec);
    if (n0 < 1 || n1 < 1 || n2 < 1 || p0 < 1 || p1 < 1)
        return set_error(MIFFT_ERR_INVALID, "grid and process grid extents must be >= 1");
    if (flags & ~(unsigned)(MIFFT_TUNE | MIFFT_PLAN_ONLY))
        return set_error(MIFFT_ERR_INVALID, "unknown flags 0x%x", flags);
    if (kind != MIFFT_C2C)
        return set_error(MIFFT_ERR_UNSUPPORTED, "the pencil share stages are C2C only");
    if (n0 % p0 || n1 % p1 || n2 % p1)
        return set_error(MIFFT_ERR_UNSUPPORTED,
                         "process grid %dx%d does not divide the %dx%dx%d grid evenly", p0, p1, n0,
                         n1, n2);
    if (!supported_length(n1) || !supported_length(n2))
        return set_error(MIFFT_ERR_UNSUPPORTED,
                         "pencil axes n1 = %d, n2 = %d must be <= 1024 with prime factors 2, 3, 5",
                         n1, n2);
    if ((long long)(n0 / p0) * (n1 / p1) >= (1LL << 31))
        return set_error(MIFFT_ERR_UNSUPPORTED, "share too large");
    int dev = 0, rc;
    const bool plan_only = flags & MIFFT_PLAN_ONLY;
    if (!plan_only && (rc = check_device(&dev))) return rc;
    mifft_plan_s* p = new mifft_plan_s();
    p->plan_only = plan_only;
    p->n0 = n0;
    p->n1 = n1;
    p->n2 = n2;
    p->p0 = p0;
    p->p1 = p1;
    p->pencil = true;
    p->kind = kind;
    p->prec = prec;
    p->device = dev;
    if (!plan_only) {
        int cus = 0;
        if (hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) == hipSuccess && cus > 0)
            p->cus = cus;
    }
    p->esz = prec == MIFFT_FP64 ? 16 : 8;
    if ((rc = build_pencil(*p, flags))) {
        delete p;
        return rc;
    }
    if (plan_only) {
        std::lock_guard<std::mutex> g(g_live_mu);
        g_live.insert(p);
        *out = static_cast<mifft_plan>(p);
        return MIFFT_OK;
    }
    return finish_plan(p, out);
}

int mifft_plan_create_slab(mifft_plan* out, int n0, int n1, int n2, int p, int kind, int prec,
                           unsigned flags)
{
    clear_error();
    if (!out) return set_error(MIFFT_ERR_INVALID, "out is NULL");
    int rc = validate_dims(n0, n1, n2, kind, prec);
    if (rc) return rc;
    if (p < 1) return set_error(MIFFT_ERR_INVALID, "task count p = %d must be >= 1", p);
    if (flags & ~(unsigned)MIFFT_PLAN_ONLY)
        return set_error(MIFFT_ERR_INVALID, "unknown flags 0x%x (slab plans take MIFFT_PLAN_ONLY only)", flags);
    if (n0 % p || n1 % p)
        return set_error(MIFFT_ERR_UNSUPPORTED, "p = %d does not divide n0 = %d and n1 = %d evenly", p, n0, n1);
    int dev = 0;
    const bool plan_only = flags & MIFFT_PLAN_ONLY;
    if (!plan_only && (rc = check_device(&dev))) return rc;
    mifft_plan_s* q = new mifft_plan_s();
    q->plan_only = plan_only;
    q->n0 = n0;
    q->n1 = n1;
    q->n2 = n2;
    q->slab = true;
    q->slab_p = p;
    q->kind = kind;
    q->prec = prec;
    q->device = dev;
    if (!plan_only) {
        int cus = 0;
        if (hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) == hipSuccess && cus > 0)
            q->cus = cus;
    }
    q->esz = prec == MIFFT_FP64 ? 16 : 8;
    if ((rc = build_slab(*q, flags))) {
        delete q;
        return rc;
    }
    if (plan_only) {
        std::lock_guard<std::mutex> g(g_live_mu);
        g_live.insert(q);
        *out = static_cast<mifft_plan>(q);
        return MIFFT_OK;
    }
    return finish_plan(q, out);
}

int mifft_plan_destroy(mifft_plan plan)
{
    clear_error();
    if (!plan) return MIFFT_OK;
    {
        std::lock_guard<std::mutex> g(g_live_mu);
        if (!g_live.erase(plan)) return set_error(MIFFT_ERR_BADPLAN, "handle is not a live plan");
    }
    delete static_cast<mifft_plan_s*>(plan);
    return MIFFT_OK;
}

const char* mifft_last_error(void) { return last_error_cstr(); }

size_t mifft_workspace_bytes(mifft_plan plan)
{
    if (!plan || !is_live(plan)) return 0;
    return (plan->pencil || plan->slab) ? 0 : plan->ws_bytes;
}

size_t mifft_poisson_ws_bytes(mifft_plan plan)
{
    if (!plan || !is_live(plan)) return 0;
    return plan->poisson_ws_bytes;
}

// The side lane of caller stream s: the one it took before, else the next
// free one of the plan's pool; nullptr when the pool is used up (the call
// then runs its list in line).  Creates nothing.  Called with p.lane_mu held.
static Plan::SideLane* side_lane(Plan& p, hipStream_t s)
{
    auto it = p.lanes.find(s);
    if (it != p.lanes.end()) return &p.lane_pool[it->second];
    if (p.lanes.size() >= p.lane_pool.size()) return nullptr;
    const int i = (int)p.lanes.size();
    p.lanes[s] = i;
    return &p.lane_pool[i];
}

// The side lanes of a plan whose pass lists have lane 1 passes (default
// priority, non-blocking streams; events without timing).
static int create_lanes(Plan& p)
{
    bool any = false;
    for (const Pass& q : p.poisson) any = any || q.lane == 1;
    if (!any) return MIFFT_OK;
    p.lane_pool.resize(Plan::kLanePool);
    for (Plan::SideLane& l : p.lane_pool) {
        hipError_t e = hipStreamCreateWithFlags(&l.s, hipStreamNonBlocking);
        if (e == hipSuccess) e = hipEventCreateWithFlags(&l.fork, hipEventDisableTiming);
        if (e == hipSuccess) e = hipEventCreateWithFlags(&l.join, hipEventDisableTiming);
        if (e != hipSuccess) return set_error(MIFFT_ERR_DEVICE, "side stream: %s", hipGetErrorString(e));
    }
    return MIFFT_OK;
}

// Launches a pass list on stream s.  With lanes_ok, passes of lane 1 run on
// a side stream of s: it starts after the lane 0 pass marked fork_after (or
// at its first lane 1 pass), and the pass marked join_before -- or the end of
// the call -- waits for it, so the call as a whole is still ordered on s.
// Per-pass timing runs every pass on s.
static int run_passes(const Plan& cp, const std::vector<Pass>& list, const void* in, void* out,
                      void* ws, void* send, void* recv, hipStream_t s, bool lanes_ok = false)
{
    Plan& p = const_cast<Plan&>(cp);
    hipEvent_t* ev = nullptr;
    if (p.prof_calls < p.prof_max_calls && (int)list.size() + 1 <= p.prof_stride) {
        ev = &p.prof_events[(size_t)p.prof_calls * p.prof_stride];
        p.prof_npass = (int)list.size();
        ++p.prof_calls;
        hipEventRecord(ev[0], s);
    }
    std::unique_lock<std::mutex> lane_lock;
    Plan::SideLane* side = nullptr;
    if (lanes_ok && !ev && std::any_of(list.begin(), list.end(), [](const Pass& q) { return q.lane == 1; })) {
        lane_lock = std::unique_lock<std::mutex>(p.lane_mu);
        side = side_lane(p, s);
    }
    bool fork_recorded = false, forked = false;
    auto join = [&]() -> hipError_t {
        forked = fork_recorded = false; // a later lane 1 pass forks anew
        hipError_t e = hipEventRecord(side->join, side->s);
        return e != hipSuccess ? e : hipStreamWaitEvent(s, side->join, 0);
    };
    int qi = 0;
    for (const Pass& q : list) {
        hipStream_t qs = s;
        if (side) {
            if (q.join_before && forked) {
                hipError_t e = join();
                if (e != hipSuccess) return set_error(MIFFT_ERR_DEVICE, "stream join: %s", hipGetErrorString(e));
            }
            if (q.lane == 1) {
                if (!forked) {
                    hipError_t e = fork_recorded ? hipSuccess : hipEventRecord(side->fork, s);
                    if (e == hipSuccess) e = hipStreamWaitEvent(side->s, side->fork, 0);
                    if (e != hipSuccess) return set_error(MIFFT_ERR_DEVICE, "stream fork: %s", hipGetErrorString(e));
                    forked = true;
                }
                qs = side->s;
            }
        }
        auto res = [&](BufId b) -> void* {
            switch (b) {
            case B_IN: return const_cast<void*>(in);
            case B_OUT: return out;
            case B_WS: return ws;
            case B_SEND: return send;
            case B_RECV: return recv;
            default: return nullptr;
            }
        };
        char* src = (char*)res(q.src);
        char* dst = (char*)res(q.dst);
        if (src) src += q.off_in;
        if (dst) dst += q.off_out;
        char* nyq = (char*)res(q.nyq_buf);
        if (q.nyq_buf != B_NONE && !nyq)
            return set_error(MIFFT_ERR_INVALID, "internal: the Nyquist plane's buffer was not provided");
        if (nyq) nyq += q.nyq_off;
        hipError_t e = launch_pass(q, p.prec, src, dst, qs, nyq);
        if (e != hipSuccess) return set_error(MIFFT_ERR_DEVICE, "kernel launch: %s", hipGetErrorString(e));
        if (ev) hipEventRecord(ev[++qi], s);
        if (side && q.fork_after && qs == s && !forked) {
            if ((e = hipEventRecord(side->fork, s)) != hipSuccess)
                return set_error(MIFFT_ERR_DEVICE, "stream fork: %s", hipGetErrorString(e));
            fork_recorded = true;
        }
    }
    if (side && forked) {
        hipError_t e = join();
        if (e != hipSuccess) return set_error(MIFFT_ERR_DEVICE, "stream join: %s", hipGetErrorString(e));
    }
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return set_error(MIFFT_ERR_DEVICE, "kernel launch: %s", hipGetErrorString(e));
    return MIFFT_OK;
}

static int check_exec(mifft_plan plan, const void* in, void* out, void* ws, bool use_ws)
{
    if (!plan) return set_error(MIFFT_ERR_INVALID, "plan is NULL");
    if (!is_live(plan)) return set_error(MIFFT_ERR_BADPLAN, "handle is not a live plan");
    if (plan->pencil)
        return set_error(MIFFT_ERR_BADPLAN, "pencil plans run through mifft_execute_pencil_stages");
    if (plan->slab) return set_error(MIFFT_ERR_BADPLAN, "slab plans run through mifft_execute_slab_stages");
    if (plan->plan_only) return set_error(MIFFT_ERR_BADPLAN, "plan was built with MIFFT_PLAN_ONLY");
    if (!in || !out) return set_error(MIFFT_ERR_INVALID, "in / out must not be NULL");
    if (!aligned16(in) || !aligned16(out))
        return set_error(MIFFT_ERR_INVALID, "in / out must be 16-byte aligned");
    if (use_ws && plan->ws_bytes && !ws)
        return set_error(MIFFT_ERR_INVALID, "this plan needs %zu bytes of workspace", plan->ws_bytes);
    if (use_ws && ws && !aligned16(ws)) return set_error(MIFFT_ERR_INVALID, "ws must be 16-byte aligned");
    if (plan->kind == MIFFT_R2C && in == out)
        return set_error(MIFFT_ERR_INVALID, "R2C / C2R must be out of place");
    return MIFFT_OK;
}

// The pass list of a call: plans with the blocked schedule run their
// transposed-schedule lists when the call is in place (in == out).
static const std::vector<Pass>& fwd_list(const Plan& p, const void* in, const void* out)
{
    return (in == out && !p.fwd_ip.empty()) ? p.fwd_ip : p.fwd;
}
static const std::vector<Pass>& inv_list(const Plan& p, const void* in, const void* out)
{
    return (in == out && !p.inv_ip.empty()) ? p.inv_ip : p.inv;
}

int mifft_execute_forward_ws(mifft_plan plan, const void* in, void* out, void* ws, void* stream)
{
    clear_error();
    int rc = check_exec(plan, in, out, ws, true);
    if (rc) return rc;
    return run_passes(*plan, fwd_list(*plan, in, out), in, out, ws, nullptr, nullptr, (hipStream_t)stream);
}

int mifft_execute_inverse_ws(mifft_plan plan, const void* in, void* out, void* ws, void* stream)
{
    clear_error();
    int rc = check_exec(plan, in, out, ws, true);
    if (rc) return rc;
    return run_passes(*plan, inv_list(*plan, in, out), in, out, ws, nullptr, nullptr, (hipStream_t)stream);
}

int mifft_execute_forward(mifft_plan plan, const void* in, void* out, void* stream)
{
    clear_error();
    int rc = check_exec(plan, in, out, nullptr, false);
    if (rc) return rc;
    return run_passes(*plan, fwd_list(*plan, in, out), in, out, plan->ws, nullptr, nullptr, (hipStream_t)stream);
}

int mifft_execute_inverse(mifft_plan plan, const void* in, void* out, void* stream)
{
    clear_error();
    int rc = check_exec(plan, in, out, nullptr, false);
    if (rc) return rc;
    return run_passes(*plan, inv_list(*plan, in, out), in, out, plan->ws, nullptr, nullptr, (hipStream_t)stream);
}

// Forward transform whose workspace is the file-scope device array below
// instead of the plan's or the caller's (for callers that cannot allocate).
// In host code `mifft_scratch` only stands for the symbol: the device address
// of each GPU's copy comes from hipGetSymbolAddress, taken once per device
// (with that device current) on the first call there, and only that address
// is ever handed to kernels.
} // extern "C"

static __device__ __align__(256) unsigned char mifft_scratch[MIFFT_SCRATCH_BYTES];

namespace {
constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
void* g_scratch_ptr[kMaxDevices] = {};
} // namespace

static int scratch_address(int dev, void** out)
{
    if (dev < 0 || dev >= kMaxDevices) return set_error(MIFFT_ERR_DEVICE, "device %d out of range", dev);
    std::lock_guard<std::mutex> g(g_scratch_mu);
    if (!g_scratch_ptr[dev]) {
        void* ptr = nullptr;
        const hipError_t e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(mifft_scratch));
        if (e != hipSuccess || !ptr)
            return set_error(MIFFT_ERR_DEVICE, "address of the static scratch array on device %d: %s", dev,
                             hipGetErrorString(e));
        g_scratch_ptr[dev] = ptr;
    }
    *out = g_scratch_ptr[dev];
    return MIFFT_OK;
}

extern "C" {

int mifft_execute_forward_static(mifft_plan plan, const void* in, void* out, void* stream)
{
    clear_error();
    if (!plan) return set_error(MIFFT_ERR_INVALID, "plan is NULL");
    if (!is_live(plan)) return set_error(MIFFT_ERR_BADPLAN, "handle is not a live plan");
    if (plan->ws_bytes > (size_t)MIFFT_SCRATCH_BYTES)
        return set_error(MIFFT_ERR_INVALID,
                         "this plan needs %zu bytes of workspace; the static scratch array holds %zu",
                         plan->ws_bytes, (size_t)MIFFT_SCRATCH_BYTES);
    int rc = check_exec(plan, in, out, nullptr, false);
    if (rc) return rc;
    int dev = -1;
    if (hipGetDevice(&dev) != hipSuccess) return set_error(MIFFT_ERR_DEVICE, "no current device");
    if (dev != plan->device)
        return set_error(MIFFT_ERR_INVALID, "the plan lives on device %d, the current device is %d", plan->device,
                         dev);
    void* ws = nullptr;
    if (plan->ws_bytes && (rc = scratch_address(dev, &ws))) return rc;
    return run_passes(*plan, fwd_list(*plan, in, out), in, out, ws, nullptr, nullptr, (hipStream_t)stream);
}

static int check_spectral(mifft_plan plan, const void* ws)
{
    if (!plan) return set_error(MIFFT_ERR_INVALID, "plan is NULL");
    if (!is_live(plan)) return set_error(MIFFT_ERR_BADPLAN, "handle is not a live plan");
    if (plan->pencil || plan->slab || plan->nd || plan->kind != MIFFT_R2C || plan->poisson_mul < 0)
        return set_error(MIFFT_ERR_BADPLAN, "spectral operators need a 3-D R2C plan");
    if (plan->plan_only) return set_error(MIFFT_ERR_BADPLAN, "plan was built with MIFFT_PLAN_ONLY");
    if (ws && !aligned16(ws)) return set_error(MIFFT_ERR_INVALID, "ws must be 16-byte aligned");
    return MIFFT_OK;
}

static int check_field(const void* p, const char* name)
{
    if (!p) return set_error(MIFFT_ERR_INVALID, "%s must not be NULL", name);
    if (!aligned16(p)) return set_error(MIFFT_ERR_INVALID, "%s must be 16-byte aligned", name);
    return MIFFT_OK;
}

static Pass renamed(Pass q, BufId from, BufId to)
{
    if (q.src == from) q.src = to;
    if (q.dst == from) q.dst = to;
    if (q.nyq_buf == from) q.nyq_buf = to;
    return q;
}

int mifft_spectral_apply(mifft_plan plan, int op, double alpha, const void* f, void* u, void* ws, void* stream)
{
    clear_error();
    int rc = check_spectral(plan, ws);
    if (rc) return rc;
    if (op < MIFFT_OP_POISSON || op > MIFFT_OP_DZ) return set_error(MIFFT_ERR_INVALID, "unknown operator %d", op);
    if ((rc = check_field(f, "f")) || (rc = check_field(u, "u"))) return rc;
    if (f == u) return set_error(MIFFT_ERR_INVALID, "f and u must not overlap");
    std::vector<Pass> list = plan->poisson;
    for (int k = 0; k < plan->poisson_mul_n; ++k) {
        list[plan->poisson_mul + k].op = op;
        list[plan->poisson_mul + k].alpha = alpha;
    }
    char* w = (char*)(ws ? ws : plan->ws);
    const size_t half = plan->poisson_ws_bytes / 2;
    // MIFFT_SIDE_STREAM=0 runs the Nyquist plane's passes in line (comparison)
    const char* e = getenv("MIFFT_SIDE_STREAM");
    const bool lanes = !(e && atoi(e) == 0);
    return run_passes(*plan, list, f, u, nullptr, w, w + half, (hipStream_t)stream, lanes);
}

int mifft_poisson_solve(mifft_plan plan, const void* f, void* u, void* ws, void* stream)
{
    return mifft_spectral_apply(plan, MIFFT_OP_POISSON, 0.0, f, u, ws, stream);
}

size_t mifft_spectral_ws_bytes(mifft_plan plan)
{
    if (!plan || !is_live(plan)) return 0;
    return plan->spectral_ws_bytes;
}

// The Poisson pass list is forward part F, multiply M, inverse part I; M
// reads and writes the buffer D that F leaves the spectrum in.  Gradient: F
// once, then per component M (D -> E, the derivative) and I (on E): E is the
// other half of the Poisson workspace where F's spectrum stays untouched by
// I, else the third buffer.  Divergence: per component F and M (D -> C, the
// third buffer, adding from the second component on), then I on C once.
int mifft_spectral_gradient(mifft_plan plan, const void* f, void* gx, void* gy, void* gz, void* ws, void* stream)
{
    clear_error();
    int rc = check_spectral(plan, ws);
    if (rc) return rc;
    if ((rc = check_field(f, "f")) || (rc = check_field(gx, "gx")) || (rc = check_field(gy, "gy")) ||
        (rc = check_field(gz, "gz")))
        return rc;
    void* g[3] = {gx, gy, gz};
    for (int j = 0; j < 3; ++j) {
        if (g[j] == f) return set_error(MIFFT_ERR_INVALID, "the outputs must not overlap f");
        for (int k = 0; k < j; ++k)
            if (g[j] == g[k]) return set_error(MIFFT_ERR_INVALID, "the outputs must be distinct");
    }
    const std::vector<Pass>& P = plan->poisson;
    const int mi = plan->poisson_mul, nm = plan->poisson_mul_n;
    const Pass& M = P[mi];
    const BufId D = M.src;
    const BufId E = M.kind == P_POISSON_X ? (D == B_SEND ? B_RECV : B_SEND) : B_WS;
    char* w = (char*)(ws ? ws : plan->ws);
    const size_t half = plan->poisson_ws_bytes / 2;
    hipStream_t s = (hipStream_t)stream;
    std::vector<Pass> fwd(P.begin(), P.begin() + mi);
    if ((rc = run_passes(*plan, fwd, f, nullptr, w + 2 * half, w, w + half, s))) return rc;
    for (int j = 0; j < 3; ++j) {
        std::vector<Pass> list;
        for (int k = 0; k < nm; ++k) { // the multiply: D -> E
            Pass m = P[mi + k];
            m.src = D;
            m.dst = E;
            m.op = MIFFT_OP_DX + j;
            m.acc = 0;
            list.push_back(m);
        }
        for (size_t k = mi + nm; k < P.size(); ++k) list.push_back(renamed(P[k], D, E));
        if ((rc = run_passes(*plan, list, nullptr, g[j], w + 2 * half, w, w + half, s))) return rc;
    }
    return MIFFT_OK;
}

int mifft_spectral_divergence(mifft_plan plan, const void* vx, const void* vy, const void* vz, void* d, void* ws,
                              void* stream)
{
    clear_error();
    int rc = check_spectral(plan, ws);
    if (rc) return rc;
    if ((rc = check_field(vx, "vx")) || (rc = check_field(vy, "vy")) || (rc = check_field(vz, "vz")) ||
        (rc = check_field(d, "d")))
        return rc;
    if (d == vx || d == vy || d == vz) return set_error(MIFFT_ERR_INVALID, "d must not overlap the inputs");
    const void* v[3] = {vx, vy, vz};
    const std::vector<Pass>& P = plan->poisson;
    const int mi = plan->poisson_mul, nm = plan->poisson_mul_n;
    const Pass& M = P[mi];
    const BufId D = M.src;
    char* w = (char*)(ws ? ws : plan->ws);
    const size_t half = plan->poisson_ws_bytes / 2;
    hipStream_t s = (hipStream_t)stream;
    for (int j = 0; j < 3; ++j) {
        std::vector<Pass> list(P.begin(), P.begin() + mi);
        for (int k = 0; k < nm; ++k) { // the multiply: D -> C (the third buffer), summed over j
            Pass m = P[mi + k];
            m.src = D;
            m.dst = B_WS;
            m.op = MIFFT_OP_DX + j;
            m.acc = j > 0;
            list.push_back(m);
        }
        if ((rc = run_passes(*plan, list, v[j], nullptr, w + 2 * half, w, w + half, s))) return rc;
    }
    std::vector<Pass> inv;
    for (size_t k = mi + nm; k < P.size(); ++k) inv.push_back(renamed(P[k], D, B_WS));
    return run_passes(*plan, inv, nullptr, d, w + 2 * half, w, w + half, s);
}

int mifft_execute_pencil_stages(mifft_plan plan, unsigned mask, void* a, void* send, void* recv,
                                void* out, void* stream)
{
    clear_error();
    if (!plan) return set_error(MIFFT_ERR_INVALID, "plan is NULL");
    if (!is_live(plan)) return set_error(MIFFT_ERR_BADPLAN, "handle is not a live plan");
    if (!plan->pencil) return set_error(MIFFT_ERR_BADPLAN, "not a pencil plan");
    if (plan->plan_only) return set_error(MIFFT_ERR_BADPLAN, "plan was built with MIFFT_PLAN_ONLY");
    const unsigned all = MIFFT_STAGE_Z | MIFFT_STAGE_PACK | MIFFT_STAGE_UNPACK | MIFFT_STAGE_Y;
    if (mask == 0 || (mask & ~all)) return set_error(MIFFT_ERR_INVALID, "bad stage mask 0x%x", mask);
    const bool z = mask & MIFFT_STAGE_Z, pk = mask & MIFFT_STAGE_PACK;
    const bool up = mask & MIFFT_STAGE_UNPACK, y = mask & MIFFT_STAGE_Y;
    auto need = [](const void* p, const char* name) {
        if (!p) return set_error(MIFFT_ERR_INVALID, "%s must not be NULL for the selected stages", name);
        if (!aligned16(p)) return set_error(MIFFT_ERR_INVALID, "%s must be 16-byte aligned", name);
        return (int)MIFFT_OK;
    };
    int rc;
    if ((z || pk) && (rc = need(a, "in"))) return rc;
    if (pk && (rc = need(send, "sendbuf"))) return rc;
    if (up && (rc = need(recv, "recvbuf"))) return rc;
    if ((up || y) && (rc = need(out, "out"))) return rc;
    std::vector<Pass> list;
    if (z && pk)
        list.push_back(plan->pz_pack);
    else if (z)
        list.push_back(plan->pz);
    else if (pk)
        list.push_back(plan->pk);
    if (up && y)
        list.push_back(plan->py_split);
    else if (up)
        list.push_back(plan->upk);
    else if (y)
        list.push_back(plan->py);
    return run_passes(*plan, list, a, out, nullptr, send, recv, (hipStream_t)stream);
}

int mifft_execute_slab_stages(mifft_plan plan, unsigned mask, const void* in, void* send, void* recv,
                              void* out, void* stream)
{
    clear_error();
    if (!plan) return set_error(MIFFT_ERR_INVALID, "plan is NULL");
    if (!is_live(plan)) return set_error(MIFFT_ERR_BADPLAN, "handle is not a live plan");
    if (!plan->slab) return set_error(MIFFT_ERR_BADPLAN, "not a slab plan");
    if (plan->plan_only) return set_error(MIFFT_ERR_BADPLAN, "plan was built with MIFFT_PLAN_ONLY");
    const bool inv = mask & MIFFT_SLAB_INVERSE;
    const unsigned st = mask & ~(unsigned)MIFFT_SLAB_INVERSE;
    const unsigned all = MIFFT_SLAB_Z | MIFFT_SLAB_Y | MIFFT_SLAB_X | (inv ? MIFFT_SLAB_UNPACK : MIFFT_SLAB_PACK);
    if (st == 0 || (st & ~all)) return set_error(MIFFT_ERR_INVALID, "bad stage mask 0x%x", mask);
    const bool z = st & MIFFT_SLAB_Z, y = st & MIFFT_SLAB_Y, x = st & MIFFT_SLAB_X;
    const bool pk = st & MIFFT_SLAB_PACK, up = st & MIFFT_SLAB_UNPACK;
    auto need = [](const void* p, const char* name) {
        if (!p) return set_error(MIFFT_ERR_INVALID, "%s must not be NULL for the selected stages", name);
        if (!aligned16(p)) return set_error(MIFFT_ERR_INVALID, "%s must be 16-byte aligned", name);
        return (int)MIFFT_OK;
    };
    int rc;
    std::vector<Pass> list;
    if (!inv) { // Z, Y (+PACK), PACK, X
        if (z && ((rc = need(in, "in")) || (rc = need(out, "out")))) return rc;
        if ((y || pk) && (rc = need(out, "out"))) return rc;
        if (pk && (rc = need(send, "sendbuf"))) return rc;
        if (x && ((rc = need(recv, "recvbuf")) || (rc = need(out, "out")))) return rc;
        if (z && in == out) return set_error(MIFFT_ERR_INVALID, "the z stage runs out of place: in != out");
        if (pk && send == out) return set_error(MIFFT_ERR_INVALID, "sendbuf must not be out");
        if (x && recv == out) return set_error(MIFFT_ERR_INVALID, "recvbuf must not be out");
        if (z) list.push_back(plan->sz);
        if (y && pk)
            list.push_back(plan->sy_pack);
        else if (y)
            list.push_back(plan->sy);
        else if (pk)
            list.push_back(plan->spk);
        if (x) list.push_back(plan->sx);
    } else { // X, UNPACK (+Y), Y, Z
        if (x && ((rc = need(in, "in")) || (rc = need(send, "sendbuf")))) return rc;
        if (up && ((rc = need(recv, "recvbuf")) || (rc = need(send, "sendbuf")))) return rc;
        if (y && (rc = need(send, "sendbuf"))) return rc;
        if (z && ((rc = need(send, "sendbuf")) || (rc = need(out, "out")))) return rc;
        if (x && in == send) return set_error(MIFFT_ERR_INVALID, "the x^-1 stage runs out of place: in != sendbuf");
        // the unpack permutes across tiles: in place only where it is the identity
        if (up && recv == send && plan->slab_p > 1)
            return set_error(MIFFT_ERR_INVALID, "recvbuf must not be sendbuf for the unpack when p > 1");
        if (z && send == out) return set_error(MIFFT_ERR_INVALID, "the z^-1 stage runs out of place: sendbuf != out");
        if (x) list.push_back(plan->sxi);
        if (up && y)
            list.push_back(plan->syi_unpack);
        else if (up)
            list.push_back(plan->supk);
        else if (y)
            list.push_back(plan->syi);
        if (z) list.push_back(plan->szi);
    }
    return run_passes(*plan, list, in, out, nullptr, send, recv, (hipStream_t)stream);
}

int mifft_profile_begin(mifft_plan plan, int max_calls)
{
    clear_error();
    if (!plan) return set_error(MIFFT_ERR_INVALID, "plan is NULL");
    if (!is_live(plan)) return set_error(MIFFT_ERR_BADPLAN, "handle is not a live plan");
    if (max_calls < 1 || max_calls > 100000) return set_error(MIFFT_ERR_INVALID, "max_calls out of range");
    size_t longest = std::max(plan->fwd.size(), std::max(plan->inv.size(), plan->poisson.size()));
    longest = std::max(longest, std::max(plan->fwd_ip.size(), plan->inv_ip.size()));
    if (longest < 4) longest = 4; // stage calls of pencil and slab plans
    const int stride = (int)longest + 1;
    const size_t need = (size_t)max_calls * stride;
    while (plan->prof_events.size() < need) {
        hipEvent_t e;
        hipError_t err = hipEventCreate(&e);
        if (err != hipSuccess) return set_error(MIFFT_ERR_DEVICE, "hipEventCreate: %s", hipGetErrorString(err));
        plan->prof_events.push_back(e);
    }
    plan->prof_stride = stride;
    plan->prof_max_calls = max_calls;
    plan->prof_calls = 0;
    plan->prof_npass = 0;
    return MIFFT_OK;
}

int mifft_profile_end(mifft_plan plan, float* avg_ms, int max_passes, int* npasses, int* ncalls)
{
    clear_error();
    if (!plan) return set_error(MIFFT_ERR_INVALID, "plan is NULL");
    if (!is_live(plan)) return set_error(MIFFT_ERR_BADPLAN, "handle is not a live plan");
    if (!avg_ms || !npasses || !ncalls || max_passes < 1) return set_error(MIFFT_ERR_INVALID, "NULL output");
    const int calls = plan->prof_calls, np = plan->prof_npass;
    *ncalls = calls;
    *npasses = np;
    for (int i = 0; i < max_passes; ++i) avg_ms[i] = 0.f;
    for (int c = 0; c < calls; ++c) {
        hipEvent_t* ev = &plan->prof_events[(size_t)c * plan->prof_stride];
        hipError_t err = hipEventSynchronize(ev[np]);
        if (err != hipSuccess) return set_error(MIFFT_ERR_DEVICE, "hipEventSynchronize: %s", hipGetErrorString(err));
        for (int i = 0; i < np && i < max_passes; ++i) {
            float ms = 0.f;
            err = hipEventElapsedTime(&ms, ev[i], ev[i + 1]);
            if (err != hipSuccess) return set_error(MIFFT_ERR_DEVICE, "hipEventElapsedTime: %s", hipGetErrorString(err));
            avg_ms[i] += ms / calls;
        }
    }
    plan->prof_max_calls = 0;
    plan->prof_calls = 0;
    return MIFFT_OK;
}

int mifft_plan_describe(mifft_plan plan, char* buf, size_t len)
{
    clear_error();
    if (!plan || !buf || len == 0) return set_error(MIFFT_ERR_INVALID, "NULL argument");
    if (!is_live(plan)) return set_error(MIFFT_ERR_BADPLAN, "handle is not a live plan");
    static const char* kn[] = {"contig", "contig_pack", "strided", "strided_unpack", "r2c_z",
                               "c2r_z",  "poisson",     "pack",    "unpack",         "copy", "poisson_x",
                               "strided_pack"};
    std::string s;
    auto add = [&](const char* tag, const Pass& q) {
        char line[640];
        int pol = q.vidx >= 0 ? variant_policy(plan->prec, q.vidx) : -1;
        int tpl = q.vidx >= 0 ? variant_tpl(plan->prec, q.vidx) : 0;
        const bool strided = q.kind == mifft::P_STRIDED || q.kind == mifft::P_STRIDED_SPLIT ||
                             q.kind == mifft::P_STRIDED_OSPLIT;
        int pf = strided && q.vidx >= 0 ? variant_prefetch(plan->prec, q.vidx) : 0;
        snprintf(line, sizeof(line),
                 "%s kind=%s axis=%c L=%d policy=%d tpl=%d sgn=%d lines=%lld lpw=%d B=%d cols=%d groups=%d "
                 "es=%lld/%lld gs=%lld/%lld off=%lld/%lld grid=%u block=%u lds=%zu pf=%d tpg=%d tiles=%d nt=%d "
                 "nto=%d gdiv=%d/%d gs2=%lld/%lld pm=%u/%lld ni=%d is=%lld/%lld os=%lld/%lld lane=%d%s%s\n",
                 tag, kn[q.kind], "zyx-"[q.tag < 3 ? q.tag : 3], q.L, pol, tpl, q.sgn, q.nlines, q.lines_per_wg,
                 q.B, q.cols, q.groups, q.es_in, q.es_out, q.gs_in, q.gs_out, q.off_in, q.off_out, q.grid,
                 q.block, q.shmem, pf, q.tpg, q.ntiles, q.nt_in, q.nt_out, q.gdiv_in, q.gdiv_out, q.gs2_in,
                 q.gs2_out, q.kind == mifft::P_CONTIG_PACK ? q.fd.d : 0u, q.kind == mifft::P_CONTIG_PACK ? q.blk : 0,
                 q.ni, q.is_o, q.is_i, q.os_o, q.os_i, q.lane, q.fork_after ? " fork=1" : "",
                 q.join_before ? " join=1" : "");
        s += line;
    };
    if (plan->pencil) {
        add("pencil_z", plan->pz);
        add("pencil_z_pack", plan->pz_pack);
        add("pencil_pack", plan->pk);
        add("pencil_unpack", plan->upk);
        add("pencil_y", plan->py);
        add("pencil_unpack_y", plan->py_split);
    } else if (plan->slab) {
        add("slab_z", plan->sz);
        add("slab_y", plan->sy);
        add("slab_y_pack", plan->sy_pack);
        add("slab_pack", plan->spk);
        add("slab_x", plan->sx);
        add("slab_x_inv", plan->sxi);
        add("slab_unpack", plan->supk);
        add("slab_y_inv", plan->syi);
        add("slab_unpack_y_inv", plan->syi_unpack);
        add("slab_z_inv", plan->szi);
    } else {
        for (const Pass& q : plan->fwd) add("forward", q);
        for (const Pass& q : plan->inv) add("inverse", q);
        for (const Pass& q : plan->poisson) add("poisson", q);
        for (const Pass& q : plan->fwd_ip) add("forward_inplace", q);
        for (const Pass& q : plan->inv_ip) add("inverse_inplace", q);
    }
    snprintf(buf, len, "%s", s.c_str());
    return MIFFT_OK;
}

const char* mifft_version(void) { return "mifft 0.1 (gfx950)"; }

int mifft_pattern_copy(int prec, const void* in, size_t in_elems, void* out, size_t out_elems, int L, int cols,
                       int groups, long long es_in, long long es_out, long long gs_in, long long gs_out, int B,
                       int threads_per_col, unsigned flags, void* stream)
{
    clear_error();
    if (prec != MIFFT_FP32 && prec != MIFFT_FP64) return set_error(MIFFT_ERR_INVALID, "bad precision %d", prec);
    if (!in || !out) return set_error(MIFFT_ERR_INVALID, "in / out must not be NULL");
    if (flags & ~(unsigned)(MIFFT_COPY_NT_LOADS | MIFFT_COPY_NT_STORES))
        return set_error(MIFFT_ERR_INVALID, "unknown flags 0x%x", flags);
    const size_t esz = prec == MIFFT_FP64 ? 16 : 8;
    if ((uintptr_t)in % esz || (uintptr_t)out % esz)
        return set_error(MIFFT_ERR_INVALID, "in / out must be aligned to the complex element");
    if (L < 1 || cols < 1 || groups < 1 || B < 1 || threads_per_col < 1 || (long long)B * threads_per_col > 1024)
        return set_error(MIFFT_ERR_INVALID, "bad tile geometry");
    if (es_in < 0 || es_out < 0 || gs_in < 0 || gs_out < 0) return set_error(MIFFT_ERR_INVALID, "negative stride");
    // one past the largest element offset read / written, in exact integer arithmetic
    const unsigned __int128 ein = (unsigned __int128)(groups - 1) * (unsigned long long)gs_in + (unsigned)(cols - 1) +
                                  (unsigned __int128)(L - 1) * (unsigned long long)es_in + 1;
    const unsigned __int128 eout = (unsigned __int128)(groups - 1) * (unsigned long long)gs_out +
                                   (unsigned)(cols - 1) + (unsigned __int128)(L - 1) * (unsigned long long)es_out + 1;
    if (ein > in_elems || eout > out_elems)
        return set_error(MIFFT_ERR_INVALID, "pattern reaches %llu / %llu elements of buffers holding %zu / %zu",
                         (unsigned long long)ein, (unsigned long long)eout, in_elems, out_elems);
    const uintptr_t a0 = (uintptr_t)in, a1 = a0 + (uintptr_t)(ein * esz);
    const uintptr_t b0 = (uintptr_t)out, b1 = b0 + (uintptr_t)(eout * esz);
    if (a0 < b1 && b0 < a1) return set_error(MIFFT_ERR_INVALID, "in and out overlap");
    hipError_t e = prec == MIFFT_FP64
                       ? launch_tile_copy<double>((const cx<double>*)in, (cx<double>*)out, L, cols, groups, B,
                                                  threads_per_col, es_in, es_out, gs_in, gs_out, flags,
                                                  (hipStream_t)stream)
                       : launch_tile_copy<float>((const cx<float>*)in, (cx<float>*)out, L, cols, groups, B,
                                                 threads_per_col, es_in, es_out, gs_in, gs_out, flags,
                                                 (hipStream_t)stream);
    if (e != hipSuccess) return set_error(MIFFT_ERR_DEVICE, "kernel launch: %s", hipGetErrorString(e));
    return MIFFT_OK;
}

int mifft_copy_reference(const void* in, void* out, size_t bytes, unsigned flags, int grid, void* stream)
{
    clear_error();
    if (!in || !out) return set_error(MIFFT_ERR_INVALID, "in / out must not be NULL");
    if (flags & ~(unsigned)(MIFFT_COPY_NT_LOADS | MIFFT_COPY_NT_STORES | MIFFT_COPY_BLOCKED))
        return set_error(MIFFT_ERR_INVALID, "unknown flags 0x%x", flags);
    if ((uintptr_t)in % 16 || (uintptr_t)out % 16 || bytes % 16)
        return set_error(MIFFT_ERR_INVALID, "pointers and size must be multiples of 16 bytes");
    if (grid < 0) return set_error(MIFFT_ERR_INVALID, "negative grid");
    const uintptr_t a0 = (uintptr_t)in, b0 = (uintptr_t)out;
    if (bytes && a0 < b0 + bytes && b0 < a0 + bytes) return set_error(MIFFT_ERR_INVALID, "in and out overlap");
    hipError_t e = launch_copy_ref(in, out, bytes, flags, grid, (hipStream_t)stream);
    if (e != hipSuccess) return set_error(MIFFT_ERR_DEVICE, "kernel launch: %s", hipGetErrorString(e));
    return MIFFT_OK;
}

int mifft_variants_describe(int prec, char* buf, size_t len)
{
    clear_error();
    if (!buf || len == 0) return set_error(MIFFT_ERR_INVALID, "NULL argument");
    if (prec != MIFFT_FP32 && prec != MIFFT_FP64) return set_error(MIFFT_ERR_INVALID, "bad precision %d", prec);
    std::string s;
    for (int i = 0; i < variant_count(prec); ++i) {
        int r[32];
        const int n = variant_radices(prec, i, r, 32);
        char line[256];
        int o = snprintf(line, sizeof(line), "L=%d policy=%d emul=%d tpl=%d radix=", variant_L(prec, i),
                         variant_policy(prec, i), variant_emul(prec, i), variant_tpl(prec, i));
        for (int k = 0; k < n && o < (int)sizeof(line) - 8; ++k) o += snprintf(line + o, sizeof(line) - o, k ? "x%d" : "%d", r[k]);
        s += line;
        s += "\n";
    }
    if (s.size() + 1 > len) return set_error(MIFFT_ERR_INVALID, "buffer of %zu bytes holds less than %zu", len, s.size() + 1);
    memcpy(buf, s.c_str(), s.size() + 1);
    return MIFFT_OK;
}

int mifft_batch_create(mifft_batch* out, int count, const int* dims, int kind, int prec, unsigned flags)
{
    clear_error();
    return batch_create(out, count, dims, kind, prec, flags);
}

int mifft_batch_execute_forward(mifft_batch batch, void* const* in, void* const* out, void* stream)
{
    clear_error();
    return batch_execute(batch, in, out, stream, false);
}

int mifft_batch_graph_launch(mifft_batch batch, void* const* in, void* const* out, void* stream)
{
    clear_error();
    return batch_execute(batch, in, out, stream, true);
}

int mifft_batch_destroy(mifft_batch batch)
{
    clear_error();
    return batch_destroy(batch);
}

int mifft_batch_check(mifft_batch batch, int* aborted)
{
    clear_error();
    return batch_check(batch, aborted);
}

int mifft_batch_describe(mifft_batch batch, char* buf, size_t len)
{
    clear_error();
    return batch_describe(batch, buf, len);
}

} // extern "C"
