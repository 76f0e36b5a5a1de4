/*
 * mifft.h -- C ABI of the MI355X-native local phases of the pencil 3-D FFT.
 *
 * The library computes, on one gfx950 GPU, the data-parallel local phases of
 * the distributed 3-D FFT of AccFFT (Gholami, Hill, Malhotra, Biros, Sec. 2,
 * Algorithm 1): batched 1-D FFTs along z, then y, then x, joined by the pack /
 * unpack steps that reshape a pencil for the row all-to-all, with R2C / C2R
 * pre- and post-processing, in single and double precision.
 *
 * Conventions (the paper leaves them open; these are the readings taken):
 *   - forward uses exp(-2 pi i jk/n), inverse exp(+2 pi i jk/n), and neither
 *     is scaled, so inverse(forward(x)) = n0*n1*n2 * x;
 *   - arrays are dense C-order [n0][n1][n2] (x slowest, z fastest) in both
 *     domains: the frequency layout equals the spatial one (Sec. 2, slab
 *     paragraph; at P0 = P1 = 1 the x-pencil and z-pencil layouts of
 *     Algorithm 1 are the same array);
 *   - complex values are interleaved (re, im): float2 / double2;
 *   - an R2C spectrum is [n0][n1][n2/2 + 1]; C2R discards the imaginary parts
 *     of its k2 = 0 and k2 = n2/2 entries (after the x and y inverses), which
 *     defines the result for input that is not Hermitian.
 *
 * Ownership: the caller owns every data, workspace and buffer pointer; a plan
 * owns its twiddle tables and its default workspace.  Every pointer passed to
 * an execute call is a device pointer on the plan's device.  Execute calls
 * only enqueue kernels on `stream` (a hipStream_t; NULL means the default
 * stream): they never allocate, synchronise or block, so they may be captured
 * into a HIP graph.  The caller must make sure no work on a plan is in flight
 * before destroying it.
 *
 * Errors: no exception crosses the ABI; every call returns an mifft_status.
 * Arguments are checked on the host before any HIP call, so argument errors
 * are reported identically with or without a GPU.  Kernel faults surface at
 * the caller's next synchronisation, as with any stream API.  The message of
 * the last failing call on the calling thread is returned by
 * mifft_last_error().  Every plan is checked when it is built: each pass's
 * reads and writes must lie inside the buffers it names (user arrays,
 * workspace); a plan that fails the check is not created
 * (MIFFT_ERR_INVALID, "internal: ...") and nothing is launched.
 *
 * Environment (read when a plan or batch is created):
 *   MIFFT_WISDOM              file of tuned choices (MIFFT_TUNE)
 *   MIFFT_CHUNK_MIB           run z / y chunk by chunk over this many MiB of planes (default 0: off)
 *   MIFFT_STRIDED_PERSIST=0   one workgroup per column tile instead of a resident grid
 *   MIFFT_PAD_ROWS=0          unpadded rows in the internal transposed intermediate
 *   MIFFT_POISSON_UNFUSED=1   Poisson solve with a standalone multiply pass
 *   MIFFT_BATCH_ITEM_KIB      data per work item of the persistent batch (default 64)
 *   MIFFT_BATCH_PUBLISH_EVERY publish batch completions after this many items (default: never early)
 * They select among equivalent schedules (for measurement); results agree
 * within rounding.
 */
#ifndef MIFFT_H
#define MIFFT_H

#include <stddef.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct mifft_plan_s* mifft_plan;   /* opaque, owned by the library */
typedef struct mifft_batch_s* mifft_batch; /* opaque, owned by the library */

typedef enum { MIFFT_C2C = 0, MIFFT_R2C = 1 } mifft_kind; /* an R2C plan also runs C2R */
typedef enum { MIFFT_FP32 = 0, MIFFT_FP64 = 1 } mifft_prec;

typedef enum {
    MIFFT_OK = 0,
    MIFFT_ERR_INVALID = 1,     /* null pointer, size < 1, bad enum, misaligned pointer */
    MIFFT_ERR_UNSUPPORTED = 2, /* prime factor > 5, odd n2 for R2C, axis too long,
                                  process grid that does not divide the grid */
    MIFFT_ERR_NOMEM = 3,       /* device allocation failed */
    MIFFT_ERR_DEVICE = 4,      /* any HIP runtime error, including "no device" */
    MIFFT_ERR_BADPLAN = 5      /* destroyed / foreign handle, or wrong plan kind */
} mifft_status;

/* Plan flags. */
#define MIFFT_HEURISTIC 0u /* kernel variants from the built-in heuristic */
#define MIFFT_TUNE 1u      /* time the candidate variants on the device and keep the
                              fastest (in the spirit of the MEASURE planning the paper
                              uses, Sec. 3, Implementation Details); consults and
                              updates the wisdom file named by MIFFT_WISDOM */

#define MIFFT_BATCH_KERNELS 4u /* batches: run the per-pass kernels of ordinary plans instead of
                                  the persistent kernel (any supported length) */
#define MIFFT_BATCH_GROUPED 8u /* batches: as MIFFT_BATCH_KERNELS, but each pass of all the
                                  transforms of one shape runs as one launch (up to 16
                                  transforms per launch; plans needing a workspace run
                                  per transform) */
#define MIFFT_PLAN_ONLY 2u /* build the pass list without touching the device: the
                              plan can be described (mifft_plan_describe) and
                              destroyed, execute calls return MIFFT_ERR_BADPLAN.
                              With MIFFT_TUNE, the choices stored in the wisdom
                              file are applied and nothing is timed; entries with
                              a tile width that is not a power of two in 1 .. 64,
                              or lines per workgroup outside 1 .. 32, are ignored */

/* Longest axis a single-pass kernel handles. */
#define MIFFT_MAX_AXIS 1024

/* Pencil stage bits for mifft_execute_pencil_stages. */
#define MIFFT_STAGE_Z 1u      /* batched z-FFT of the local share (Algorithm 1) */
#define MIFFT_STAGE_PACK 2u   /* pack into the row all-to-all send layout (Sec. 2) */
#define MIFFT_STAGE_UNPACK 4u /* unpack the receive layout (Sec. 2) */
#define MIFFT_STAGE_Y 8u      /* batched y-FFT (Algorithm 1) */

/*
 * mifft_plan_create -- plan a 3-D transform of an n0 x n1 x n2 grid.
 * Defines: the problem statement of Sec. 1 (Contributions: an N0 x N1 x N2
 * array, R2C / C2C / C2R, single and double precision).
 *   out    receives the handle (unchanged on error)
 *   n0..2  grid extents, each 1 .. MIFFT_MAX_AXIS with no prime factor above 5;
 *          R2C needs an even n2
 *   kind   MIFFT_C2C or MIFFT_R2C (the R2C plan runs C2R as its inverse)
 *   prec   MIFFT_FP32 (complex64 / float32) or MIFFT_FP64
 *   flags  MIFFT_HEURISTIC, MIFFT_TUNE or MIFFT_PLAN_ONLY
 * Allocates device twiddle tables (generated in FP64 on the GPU, rounded to
 * nearest for FP32 plans) and the default workspace on the current device.
 */
int mifft_plan_create(mifft_plan* out, int n0, int n1, int n2, int kind, int prec,
                      unsigned flags);

/*
 * mifft_execute_forward -- forward transform (Algorithm 1, left column:
 * z-FFT, y-FFT, x-FFT; at P0 = P1 = 1 both exchanges are identities).
 *   C2C: in, out complex [n0][n1][n2]; in == out is allowed.
 *   R2C: in real [n0][n1][n2], out complex [n0][n1][n2/2+1]; must not overlap.
 * `in` is not modified unless in == out.  Uses the plan's default workspace.
 */
int mifft_execute_forward(mifft_plan plan, const void* in, void* out, void* stream);

/*
 * mifft_execute_inverse -- unscaled inverse transform (Algorithm 1, right
 * column: x-IFFT, y-IFFT, z-IFFT).
 *   C2C: in, out complex [n0][n1][n2]; in == out is allowed.
 *   C2R: in complex [n0][n1][n2/2+1], out real [n0][n1][n2]; must not overlap;
 *        `in` is preserved (the intermediate lives in the workspace).
 */
int mifft_execute_inverse(mifft_plan plan, const void* in, void* out, void* stream);

/* Bytes of workspace an execute call of this plan needs (0 if none). */
size_t mifft_workspace_bytes(mifft_plan plan);

/* As above with a caller-owned workspace of at least mifft_workspace_bytes
 * bytes (NULL when that is 0).  Two execute calls of one plan may run
 * concurrently on different streams only through these variants, each with
 * its own workspace; the plain variants share the plan's default one. */
int mifft_execute_forward_ws(mifft_plan plan, const void* in, void* out, void* ws,
                             void* stream);
int mifft_execute_inverse_ws(mifft_plan plan, const void* in, void* out, void* ws,
                             void* stream);

/*
 * mifft_execute_forward_static -- for callers that cannot allocate (code
 * under HIP graph capture, tight serving loops, harnesses that forbid
 * hipMalloc): mifft_execute_forward with its workspace in a file-scope
 * device array of MIFFT_SCRATCH_BYTES that the library holds on every GPU
 * it runs on until the process ends.  The call allocates nothing (no
 * hipMalloc / hipFree, no allocating library routine); the caller passes
 * `in` and `out` as for mifft_execute_forward.
 *   Errors: MIFFT_ERR_INVALID when the plan's workspace
 *   (mifft_workspace_bytes) exceeds MIFFT_SCRATCH_BYTES (checked before any
 *   HIP call) or when the current device is not the plan's; otherwise as
 *   mifft_execute_forward.
 *   Concurrency: every call on one GPU shares that GPU's array, so calls
 *   that overlap on one GPU (other streams, other threads) race; nothing in
 *   the array needs to start at zero.
 */
#define MIFFT_SCRATCH_BYTES (256u << 20)
int mifft_execute_forward_static(mifft_plan plan, const void* in, void* out, void* stream);

/*
 * mifft_plan_destroy -- free the plan's device memory.  NULL is a no-op that
 * returns MIFFT_OK; a handle that is not live returns MIFFT_ERR_BADPLAN.
 */
int mifft_plan_destroy(mifft_plan plan);

/* Message of the last failing call on this thread ("" if none).  The pointer
 * stays valid until the next mifft call on the same thread. */
const char* mifft_last_error(void);

/*
 * mifft_plan_create_nd -- plan a transform of a C-order array of any rank
 * 1 .. MIFFT_MAX_RANK (Algorithm 2 with one task per axis: batched 1-D FFTs
 * along the last axis, then along each earlier axis in turn; the inverse in
 * the opposite order).  dims[0] is the slowest extent, dims[rank-1] the
 * contiguous one; R2C halves the last axis to dims[rank-1]/2 + 1.  Rank 1 .. 3
 * is the 3-D plan of mifft_plan_create with leading extents of 1 (all its
 * flags apply); rank >= 4 takes MIFFT_PLAN_ONLY only (MIFFT_TUNE:
 * UNSUPPORTED) and has at most 2^31 - 1 elements.  Execute with
 * mifft_execute_forward / _inverse (and the _ws variants); the C2R inverse
 * keeps its input (its complex passes run in the workspace).  The Poisson
 * solve needs a rank-3 plan.  Errors as mifft_plan_create, plus INVALID for
 * a NULL dims or a rank outside 1 .. MIFFT_MAX_RANK.
 */
#define MIFFT_MAX_RANK 8
int mifft_plan_create_nd(mifft_plan* out, int rank, const int* dims, int kind, int prec, unsigned flags);

/*
 * mifft_plan_create_pencil -- plan one rank's share of the pencil-decomposed
 * forward transform of an N0 x N1 x N2 C2C grid on a p0 x p1 process grid
 * (Sec. 2, pencil paragraph; Algorithm 1, up to the y-FFT).  The share is the
 * local array A[N0/p0][N1/p1][N2]; with M = N2/p1 the stages compute
 *   Z:      Ahat = z-FFT of A along its last axis (length N2)
 *   PACK:   S[j][i0][i1][m] = Ahat[i0][i1][j*M + m]   (send block j -> row peer j)
 *   UNPACK: B[i0][j*(N1/p1) + i1][m] = R[j][i0][i1][m] (R = receive buffer)
 *   Y:      y-FFT of B along its middle axis (length N1)
 * The row all-to-all between PACK and UNPACK is not performed here: on one
 * GPU the caller passes recvbuf == sendbuf (loopback) or moves the blocks
 * itself.  Needs kind = MIFFT_C2C and N0 % p0 == N1 % p1 == N2 % p1 == 0.
 */
int mifft_plan_create_pencil(mifft_plan* out, int n0, int n1, int n2, int p0, int p1,
                             int kind, int prec, unsigned flags);

/*
 * mifft_execute_pencil_stages -- run the stages named in stage_mask, in the
 * order Z, PACK, UNPACK, Y.  Buffers (all complex, dense):
 *   in       A, (N0/p0) x (N1/p1) x N2           read by Z (or by PACK without Z);
 *                                                Z without PACK overwrites it
 *   sendbuf  S, p1 x (N0/p0) x (N1/p1) x M       written by PACK
 *   recvbuf  R, same shape as S                  read by UNPACK
 *   out      B, (N0/p0) x N1 x M                 written by UNPACK, transformed by Y
 * Z without PACK writes Ahat to `in` in place; Z with PACK writes S directly
 * (pack fused into the z-FFT's stores).  UNPACK with Y reads R directly
 * (unpack fused into the y-FFT's loads).  Y without UNPACK transforms `out`
 * in place.  Buffers a selected stage does not touch may be NULL.
 */
int mifft_execute_pencil_stages(mifft_plan plan, unsigned stage_mask, void* in,
                                void* sendbuf, void* recvbuf, void* out, void* stream);

/*
 * mifft_plan_create_slab -- plan one task's share of the slab-decomposed
 * transform of an N0 x N1 x N2 grid over p tasks (Algorithm 3; Sec. 2, slab
 * paragraph), C2C or R2C / C2R, FP32 or FP64.  With n0l = N0/p, n1l = N1/p
 * and N2c = N2 (C2C) or N2/2 + 1 (R2C):
 *   spatial slab    A[n0l][N1][N2]     (real for R2C), x rows r n0l ... of task r
 *   spectral share  X[N0][n1l][N2c]    y rows r n1l ... of task r
 *   send / receive  S, R[p][n0l][n1l][N2c]: block j goes to / came from task j
 * The complex buffers (out, sendbuf, recvbuf, and `in` of the inverse) all
 * hold n0l N1 N2c = N0 n1l N2c elements.  Forward stages, in this order:
 *   Z:    2-D FFT part 1, z-FFT (R2C) of A: in -> out            (in kept)
 *   Y:    2-D FFT part 2, y-FFT: in place on out; with PACK its
 *         stores go straight to the send layout out -> sendbuf,
 *         S[j][i0][i1][k2] = Ahat[i0][j n1l + i1][k2]
 *   PACK: without Y, the same map as a copy out -> sendbuf
 *   X:    x-FFT of the received slab recvbuf -> out, where the block
 *         from task s supplies x rows s n0l ... (no unpack needed)
 * Inverse stages (mask | MIFFT_SLAB_INVERSE), in this order:
 *   X:      x-IFFT of X: in -> sendbuf, whose block r (x rows r n0l ...)
 *           is already contiguous
 *   UNPACK: A[i0][s n1l + i1][k2] = R[s][i0][i1][k2]: recvbuf -> sendbuf;
 *           with Y fused into the y-IFFT's loads
 *   Y:      y-IFFT: in place on sendbuf (without UNPACK)
 *   Z:      z-IFFT (C2R for R2C plans, imaginary parts of k2 = 0 and N2/2
 *           discarded): sendbuf -> out; sendbuf is kept
 * Unscaled in both directions.  The all-to-all between the halves is not
 * performed here: with p = 1 the caller passes recvbuf == sendbuf
 * (loopback), otherwise it moves the blocks itself.  Errors: p must divide
 * N0 and N1 (UNSUPPORTED); the out-of-place stages reject aliased buffers
 * and an unpack with recvbuf == sendbuf when p > 1 (INVALID).  Flags:
 * MIFFT_PLAN_ONLY only.  No workspace.
 */
#define MIFFT_SLAB_Z 1u
#define MIFFT_SLAB_Y 2u
#define MIFFT_SLAB_X 4u
#define MIFFT_SLAB_PACK 8u       /* forward only */
#define MIFFT_SLAB_UNPACK 16u    /* inverse only */
#define MIFFT_SLAB_INVERSE 256u  /* selects the inverse stages */
int mifft_plan_create_slab(mifft_plan* out, int n0, int n1, int n2, int p, int kind, int prec,
                           unsigned flags);
int mifft_execute_slab_stages(mifft_plan plan, unsigned stage_mask, const void* in, void* sendbuf,
                              void* recvbuf, void* out, void* stream);

/*
 * mifft_poisson_solve -- periodic Poisson solve lap(u) = f on [0, 2 pi)^3
 * with an R2C plan: R2C forward, multiply the half spectrum by
 * -1 / (|k|^2 n0 n1 n2) with the k = 0 mode set to zero (signed wavenumbers
 * k' = k for k < n/2, else k - n, along x and y), C2R inverse.  One of the
 * "fast spectral operators" listed in Sec. 1.  f and u are real
 * [n0][n1][n2]; ws is a caller-owned workspace of mifft_poisson_ws_bytes
 * bytes, or NULL to use the plan's default one (then calls on one plan must
 * not overlap).  f is preserved; f and u must not overlap.
 */
size_t mifft_poisson_ws_bytes(mifft_plan plan);
int mifft_poisson_solve(mifft_plan plan, const void* f, void* u, void* ws, void* stream);

/*
 * Spectral operators on the periodic box [0, 2 pi)^3 with a 3-D R2C plan
 * (more of the "fast spectral operators" listed in Sec. 1): u = C2R(m(k) *
 * R2C(f)) / (n0 n1 n2), with integer wavenumbers k0 = i0 below n0/2, else
 * i0 - n0 (likewise k1), k2 = i2:
 *   MIFFT_OP_POISSON    -1/|k|^2, 0 at k = 0 (u solves lap(u) = f; as
 *                       mifft_poisson_solve)
 *   MIFFT_OP_LAPLACIAN  -|k|^2 (u = lap(f))
 *   MIFFT_OP_HELMHOLTZ  1/(alpha + |k|^2), 0 where that vanishes (u solves
 *                       alpha u - lap(u) = f)
 *   MIFFT_OP_DX/DY/DZ   i k_j (u = df/dx_j); on an even axis the Nyquist
 *                       mode i_j = n_j/2 is set to 0
 * The x-forward, the multiply and the x-inverse run as one kernel (for
 * n0 > 1).  f, u and the outputs below are real [n0][n1][n2] device arrays;
 * f is preserved; outputs must not overlap inputs.  ws: NULL (the plan's
 * own workspace; calls on one plan must then not overlap) or a caller buffer
 * of mifft_poisson_ws_bytes (apply) or mifft_spectral_ws_bytes (gradient,
 * divergence) bytes.  Errors: BADPLAN for a plan that is not a 3-D R2C
 * plan, INVALID for NULL / unaligned / aliased fields or an unknown op.
 * On plans whose half spectrum is 256 MiB or more, mifft_spectral_apply and
 * mifft_poisson_solve run the k2 = n2/2 plane's passes on a side stream that
 * the plan created with itself (one of four, taken by a caller stream at its
 * first such call and kept): it waits for `stream`, and `stream` waits for
 * it before the last pass, so the call is still ordered on `stream` and may
 * be captured.  Calls on a fifth distinct stream run those passes on
 * `stream` itself.
 */
#define MIFFT_OP_POISSON 0
#define MIFFT_OP_LAPLACIAN 1
#define MIFFT_OP_HELMHOLTZ 2
#define MIFFT_OP_DX 3
#define MIFFT_OP_DY 4
#define MIFFT_OP_DZ 5
int mifft_spectral_apply(mifft_plan plan, int op, double alpha, const void* f, void* u, void* ws, void* stream);
size_t mifft_spectral_ws_bytes(mifft_plan plan);
/* (df/dx, df/dy, df/dz): one forward transform, then per component the
 * fused multiply and the inverse. */
int mifft_spectral_gradient(mifft_plan plan, const void* f, void* gx, void* gy, void* gz, void* ws,
                            void* stream);
/* dvx/dx + dvy/dy + dvz/dz: per component the forward transform and the fused
 * multiply, summed in the spectrum; then one inverse. */
int mifft_spectral_divergence(mifft_plan plan, const void* vx, const void* vy, const void* vz, void* d,
                              void* ws, void* stream);

/*
 * mifft_batch_create -- plan `count` (1 .. 128) independent 3-D C2C transforms
 * of uneven sizes (dims holds n0, n1, n2 per transform) that run as ONE
 * launch of a persistent kernel: workgroups pull (transform, pass, tile)
 * work items from a device queue in dependency order (all z-passes, then all
 * y-passes, then all x-passes; a pass waits on a completion counter of the
 * previous pass of its transform).  Every axis length must be 2 .. 256 with
 * prime factors 2, 3, 5, unless MIFFT_BATCH_KERNELS asks for the per-pass
 * kernels of ordinary plans instead, or MIFFT_BATCH_GROUPED for those kernels
 * with one launch per pass and shape (then MIFFT_TUNE tunes those plans).
 * The batched local FFTs are the per-task work of Alg. 1 for many grids at
 * once; scheduling them as one launch is this library's own design.
 */
int mifft_batch_create(mifft_batch* out, int count, const int* dims, int kind, int prec,
                       unsigned flags);

/* Forward transforms of the whole batch: in[t], out[t] are device pointers
 * to complex [n0][n1][n2] arrays; in[t] == out[t] is allowed.  The pointer
 * arrays are host arrays read during the call. */
int mifft_batch_execute_forward(mifft_batch batch, void* const* in, void* const* out,
                                void* stream);

/* Capture one mifft_batch_execute_forward with these buffers into a HIP
 * graph owned by the batch, then launch the instantiated graph on `stream`.
 * Later calls with the same pointer arrays replay the graph. */
int mifft_batch_graph_launch(mifft_batch batch, void* const* in, void* const* out,
                             void* stream);

int mifft_batch_destroy(mifft_batch batch);

/* Waits for the device and reports in *aborted whether any bounded wait of
 * the persistent kernel ran out (1) since the last launch, in which case the
 * outputs of that launch are not valid; 0 otherwise. */
int mifft_batch_check(mifft_batch batch, int* aborted);

/* Writes a one-line description of the batch (mode, passes, work items,
 * persistent grid, LDS) into buf. */
int mifft_batch_describe(mifft_batch batch, char* buf, size_t len);

/*
 * Introspection for tests, benchmarks and the autotuner.
 * mifft_plan_describe writes a NUL-terminated description of the passes of
 * the plan (kernel variant, length, stride, batch, launch shape), one line
 * per pass, into buf (at most len bytes) and returns MIFFT_OK.
 */
int mifft_plan_describe(mifft_plan plan, char* buf, size_t len);

/*
 * Per-pass timing for benchmarks (the per-phase breakdown of Sec. 3, Fig. 3e-f
 * and Fig. 4, on the local phases).  mifft_profile_begin makes the next
 * `max_calls` execute calls of this plan record a HIP event on their stream
 * before the first pass and after every pass.  mifft_profile_end waits for
 * those events, writes the mean duration in milliseconds of each pass of the
 * most recent pass list (at most max_passes values) into avg_ms, their count
 * into *npasses and the number of profiled calls into *ncalls, and stops
 * recording.  Calls beyond max_calls are not recorded.  Event records cost a
 * few microseconds per pass and are captured like any other stream work.
 */
int mifft_profile_begin(mifft_plan plan, int max_calls);
int mifft_profile_end(mifft_plan plan, float* avg_ms, int max_passes, int* npasses, int* ncalls);

/* Version string of the library build. */
const char* mifft_version(void);

/* Measurement references (flags: MIFFT_COPY_NT_LOADS / MIFFT_COPY_NT_STORES
 * select streaming loads / stores, as the FFT passes use them).
 *
 * mifft_pattern_copy copies complex elements with the access pattern of a
 * strided pass and no arithmetic -- for group g < groups, column c < cols
 * and row r < L, out[g*gs_out + c + r*es_out] = in[g*gs_in + c + r*es_in]
 * (strides in complex elements), in tiles of B columns x L rows with
 * threads_per_col threads per column.  Its rate is the ceiling of that access
 * pattern on the device, against which a strided FFT pass's bandwidth is
 * read.  The caller owns both buffers; in_elems / out_elems are their sizes
 * in complex elements.  INVALID, before anything is launched, for NULL
 * pointers, pointers not aligned to the element, a non-positive extent,
 * B x threads_per_col > 1024, a negative stride, unknown flags, offsets
 * reaching past in_elems / out_elems, or overlapping source and destination
 * ranges. */
#define MIFFT_COPY_NT_LOADS 1u
#define MIFFT_COPY_NT_STORES 2u
#define MIFFT_COPY_BLOCKED 4u
int mifft_pattern_copy(int prec, const void* in, size_t in_elems, void* out, size_t out_elems, int L, int cols,
                       int groups, long long es_in, long long es_out, long long gs_in, long long gs_out, int B,
                       int threads_per_col, unsigned flags, void* stream);

/* mifft_copy_reference copies `bytes` (a multiple of 16) from in to out with
 * 16-byte vector accesses, several in flight per thread, over `grid`
 * workgroups of 256 threads (0: enough for four words per thread) -- the
 * plain contiguous copy, the achievable bandwidth ceiling of the device.
 * With MIFFT_COPY_BLOCKED each workgroup of 128 threads copies one
 * contiguous 8 KiB block, all its loads before its stores (the grid is then
 * the number of blocks; `grid` is ignored).
 * Both buffers hold at least `bytes` and are caller-owned.  INVALID for NULL
 * or unaligned pointers, a size not a multiple of 16, a negative grid,
 * unknown flags or overlapping ranges. */
int mifft_copy_reference(const void* in, void* out, size_t bytes, unsigned flags, int grid, void* stream);

/* One line per compiled kernel variant of a precision -- the autotuner's
 * search space (the candidates MIFFT_TUNE times, in the spirit of the MEASURE
 * planning of Sec. 3): "L=<length> policy=<radix order> emul=<radix groups
 * per thread> tpl=<threads per line> radix=<r1>x<r2>x..." (stage order).
 * Needs no device.  INVALID if buf is NULL, shorter than the text, or prec
 * is not MIFFT_FP32 / MIFFT_FP64. */
int mifft_variants_describe(int prec, char* buf, size_t len);

#ifdef __cplusplus
}
#endif

#endif /* MIFFT_H */
