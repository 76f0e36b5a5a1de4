// plan.hpp -- host-side plan: the pass list of one transform and its launch
// geometry, shared by the single-transform C ABI and the batched executor.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdarg>
#include <cstdint>
#include <map>
#include <mutex>
#include <string>
#include <vector>

#include "../../include/mifft.h"
#include "registry.hpp"

namespace mifft {

enum PassKind {
    P_CONTIG = 0,
    P_CONTIG_PACK,
    P_STRIDED,
    P_STRIDED_SPLIT,
    P_R2C,
    P_C2R,
    P_POISSON,
    P_PACK,
    P_UNPACK,
    P_COPY,
    P_POISSON_X, // fused x-forward, Poisson multiply, x-inverse (in place)
    P_STRIDED_OSPLIT // strided pass storing through a split (slab pack) map
};

// Which caller buffer a pass reads or writes; resolved at execute time.
enum BufId { B_NONE = 0, B_IN, B_OUT, B_WS, B_SEND, B_RECV };

struct Pass {
    PassKind kind = P_COPY;
    int L = 1;
    int vidx = -1; // index into the variant table of the plan's precision
    BufId src = B_NONE, dst = B_NONE;
    int sgn = 1;   // +1 forward, -1 inverse
    // contiguous / real passes: line l at (l / ni) * s_o + (l % ni) * s_i
    long long nlines = 0;
    int lines_per_wg = 1;
    int ni = 1;
    long long is_o = 0, is_i = 0, os_o = 0, os_i = 0;
    // strided passes
    int B = 1, log2B = 0, cols = 0, ntiles = 0, groups = 0;
    int tpg = 0; // tiles per group; 0: tiles over the flattened (group, column) index
    int nt_in = 0; // strided: streaming loads (tiles read whole, aligned 128-byte lines)
    int nt_out = 0; // R2C / C2R z-pass: streaming stores (set by make_real_z from the output size)
    long long gs_in = 0, gs_out = 0, es_in = 0, es_out = 0;
    // two-level group maps (blocked layouts): with gdiv > 1, group g at
    // (g / gdiv) gs + (g % gdiv) gs2 on that side
    int gdiv_in = 0, gdiv_out = 0;
    long long gs2_in = 0, gs2_out = 0;
    int fixedB = 0; // the layout fixes the tile width (a blocked intermediate): the tuner keeps it
    // R2C / C2R z-pass: element n2/2 of line (lo, li) at nyq_buf + nyq_off
    // (bytes) + (lo nyq_o + li nyq_i) elements, a plane of its own
    BufId nyq_buf = B_NONE;
    long long nyq_off = 0, nyq_o = 0, nyq_i = 0;
    int k2_fixed = -1; // fused spectral x-pass over one k2 plane [x][k1]: every column is (k1, k2_fixed)
    // pack / split
    FastDiv fd{1, 1ull << 32};
    long long blk = 0;
    // auxiliary kernels
    int n0 = 0, n1 = 0, n2c = 0, p1 = 0, M = 0;
    // spectral multiply (P_POISSON, P_POISSON_X): operator, its parameter,
    // the full z length (Nyquist index), and whether to add to the output
    int op = 0, nz = 0, acc = 0;
    double alpha = 0.0;
    size_t bytes = 0;
    double scale = 1.0;
    // byte offsets added to the resolved source / destination (chunked passes)
    long long off_in = 0, off_out = 0;
    int tag = 0; // 0 z, 1 y, 2 x, 3 other: for per-axis timing summaries
    // Concurrency within a pass list (see run_passes): lane 1 passes may run on
    // a side stream, after the lane 0 pass marked fork_after (or from the
    // start of the call); a pass marked join_before waits for them.
    int lane = 0;
    bool fork_after = false, join_before = false;
    // launch geometry
    unsigned grid = 0, block = 0;
    size_t shmem = 0;
    const void* tw = nullptr;
    const void* tw2 = nullptr;
};

struct TuneChoice {
    int contig = -1; // variant index per axis kind, -1 = heuristic
    int strided = -1;
};

class Plan {
public:
    int n0 = 1, n1 = 1, n2 = 1, kind = MIFFT_C2C, prec = MIFFT_FP32;
    // The y-pass writes a transposed intermediate W[ky][x][k2] into the
    // workspace so that the x-pass reads with a small stride (see plan.hip).
    bool transposed = false;
    int ncw = 0; // row pitch (complex elements) of the internal k2 rows: nc rounded up to 128 bytes
    bool plan_only = false; // no device resources: describe only
    int chunks = 1;         // z/y (forward) and x/z (inverse) interleaved in this many chunks
    bool pencil = false;
    int p0 = 1, p1 = 1;
    int device = 0;
    int cus = 256;  // compute units of the device (persistent grids)
    size_t esz = 8; // bytes per complex element
    std::vector<Pass> fwd, inv, poisson;
    // With the blocked schedule (out of place only), fwd / inv pass through
    // blocked intermediates; an in-place call (in == out) runs these lists,
    // the transposed schedule, instead.  Empty otherwise.
    std::vector<Pass> fwd_ip, inv_ip;
    int blocked = 0; // block width (columns) of the blocked intermediates, 0: not used
    // pencil stages
    Pass pz, pz_pack, pk, upk, py, py_split;
    // slab stages (Algorithm 3) of one of slab_p tasks: forward z, y, y with
    // the pack fused, standalone pack, x; inverse x, standalone unpack, y,
    // y with the unpack fused, z
    bool slab = false;
    int slab_p = 1;
    // arrays of rank > 3 (Algorithm 2): the extents, first (slowest) to last;
    // n0 n1 n2 then hold (product of the leading extents, second-to-last, last)
    bool nd = false;
    std::vector<int> dims;
    Pass sz, sy, sy_pack, spk, sx, sxi, supk, syi, syi_unpack, szi;
    std::map<int, void*> twiddles; // length -> device table
    void* ws = nullptr;
    size_t ws_bytes = 0;         // workspace an execute call needs
    size_t default_ws_bytes = 0; // size of the plan's own workspace (covers Poisson too)
    size_t poisson_ws_bytes = 0;  // two half-spectrum buffers (Poisson solve, one operator)
    size_t spectral_ws_bytes = 0; // three (gradient, divergence)
    int poisson_mul = -1;         // index of the multiply pass in `poisson`
    int poisson_mul_n = 1;        // multiply passes from there (2 with the Nyquist plane on its own)
    // opt-in per-pass event timing
    std::vector<hipEvent_t> prof_events; // max_calls * (max passes + 1)
    int prof_max_calls = 0, prof_calls = 0, prof_stride = 0, prof_npass = 0;
    // side streams of the lane 1 passes with the fork and join events of each,
    // created with the plan (kLanePool of them where a pass list has lane 1
    // passes); a caller stream takes one at its first such call and keeps it
    struct SideLane {
        hipStream_t s = nullptr;
        hipEvent_t fork = nullptr, join = nullptr;
    };
    static constexpr int kLanePool = 4;
    std::vector<SideLane> lane_pool;
    std::map<hipStream_t, int> lanes; // caller stream -> index into lane_pool
    std::mutex lane_mu;

    ~Plan();
};

// Status helpers (thread-local last error message).
int set_error(int status, const char* fmt, ...);
void clear_error();

// Variant table access for the plan's precision.
int variant_count(int prec);
int variant_L(int prec, int idx);
int variant_tpl(int prec, int idx);
int variant_policy(int prec, int idx);
int variant_emul(int prec, int idx);
int variant_prefetch(int prec, int idx);
int variant_poisson_B(int prec, int idx);
void set_tile_width(Pass& p, int prec, int tpl, int B);
int variant_radices(int prec, int idx, int* radix, int max); // stage count; radices in stage order
int find_variant(int prec, int L, int policy, int emul);
int default_variant(int prec, int L);
int contig_variant(int prec, int L);

bool supported_length(int L);
FastDiv make_fastdiv(uint32_t d);

// Launch geometry heuristics.
void set_contig_geometry(Pass& p, int prec, int tpl, int L, long long nlines, int lds_len);
// Grid of a strided pass whose tile shape is set: one workgroup per tile, or,
// for kernels that prefetch their next tile, at most as many workgroups as
// the device holds at once (each then walks tiles with the grid's stride).
void strided_grid(const Plan& plan, Pass& p);
// Tiling of a strided / fused-Poisson pass whose strides and tile width are
// set: tiles over the flattened (group, column) index where either side is
// contiguous across groups (gs = cols), else per group; then its grid.
void tile_pass(const Plan& plan, Pass& p);
void tile_passes(Plan& plan);
// Every pass's reads and writes stay inside its buffers (MIFFT_OK), or an
// internal error is set and returned.
int validate_extents(const Plan& plan);
// Largest element offset (plus one) a pass reads and writes, including its
// byte offsets; complex elements (pairs of reals on the real side).
struct Extent {
    long long in, out;
};
Extent pass_extent(const Pass& p, size_t esz);
void set_line_map(Pass& p, int ni, long long is_o, long long is_i, long long os_o, long long os_i);
void set_strided_geometry(Pass& p, int prec, int tpl, int L, int cols, int groups, int forceB);

// Enqueue one pass with resolved buffers.
// `nyq`: the resolved nyq_buf + nyq_off of the pass, if it has one.
hipError_t launch_pass(const Pass& p, int prec, const void* src, void* dst, hipStream_t s, void* nyq = nullptr);
// The same contiguous or strided pass of ng <= kMaxGroup transforms of one
// shape as one launch (member i: src[i] -> dst[i]).
hipError_t launch_pass_group(const Pass& p, int prec, int ng, const void* const* src, void* const* dst,
                             hipStream_t s);
// The plan behind a C-ABI handle (no liveness check).
const Plan* plan_of(mifft_plan h);

// Generate (or reuse) the twiddle table of length L on the current device.
int get_twiddles(Plan& plan, int L, void** out);

int build_plan(Plan& plan, unsigned flags);
// wisdom entries of the batched executor (tune.hip): [policy, emul, item KiB, microseconds]
bool wisdom_batch_get(const std::string& key, int* policy, int* emul, int* item_kib);
void wisdom_batch_put(const std::vector<std::pair<std::string, std::vector<double>>>& entries);
void rebuild_poisson(Plan& plan); // re-derive the Poisson pass list from fwd / inv
void apply_chunking(Plan& plan);  // interleave z/y (x^-1/z^-1) over plane chunks
int build_pencil(Plan& plan, unsigned flags);
int build_slab(Plan& plan, unsigned flags);
int build_nd(Plan& plan, unsigned flags);

} // namespace mifft
