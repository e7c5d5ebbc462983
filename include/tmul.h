/*
 * tmul.h - truncated integer multiplication on AMD Instinct MI355X (gfx950).
 *
 * Implements the hot path of D. Harvey, "Faster truncated integer
 * multiplication" (arXiv 1703.00640): the low product uv mod 2^n and the high
 * product (the top n bits of uv, possibly one too large) of two n-bit
 * integers through a real cyclic convolution of length N, instead of the
 * length 2N that the full 2n-bit product needs (Algorithms "low product" and
 * "high product"), and the full product itself (Algorithm "full product").
 *
 * Conventions for every entry point
 * ---------------------------------
 * - Integers are little-endian arrays of uint64_t limbs in DEVICE memory.
 *   An n-bit operand has L = ceil(n/64) limbs; bits at positions >= n are
 *   ignored (the library masks them).
 * - Outputs: low and high product -> L limbs, bits >= n cleared; full
 *   product -> 2L limbs.
 * - The caller owns u, v, w and the workspace.  w must not overlap u, v or
 *   the workspace.  u == v (the same pointer) computes a square with one
 *   forward transform instead of two.  Workspace size comes from
 *   tm_workspace_bytes() and must be at least that many bytes, 256-byte
 *   aligned.
 * - All calls are asynchronous on the given HIP stream (NULL = default
 *   stream) and do not synchronise, except tm_mul_checked().  Two calls may
 *   run concurrently only with distinct workspaces.
 * - Errors are reported through the return code only; nothing is thrown and
 *   nothing exits.  After TM_ERR_HIP, tm_last_error() describes the failing
 *   HIP call (per thread).
 * - Graph capture: tm_mul and its wrappers launch kernels only, so they can
 *   be captured into a HIP graph (stream capture) once the size's tables
 *   exist (tm_prepare, or one earlier call); a call that would have to
 *   build them during a capture returns TM_ERR_INVALID.  Replays read the
 *   captured buffers' current contents.  tm_mul_batched / tm_mul_packed
 *   upload metadata from a reused host buffer and are not for capture.
 * - The library keeps one device-side cache per (device, transform length):
 *   the FFT twiddle tables, built on first use (this first call synchronises
 *   its stream once), and a few pinned host buffers for the launch metadata
 *   of packed batches.  tm_release_caches() waits for all work on the devices
 *   holding tables (hipDeviceSynchronize) and frees them.
 */
#ifndef TMUL_H
#define TMUL_H

#include <stddef.h>
#include <stdint.h>
#include <hip/hip_runtime_api.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
    TM_FULL = 0, /* uv                                   (Algorithm full)  */
    TM_LO = 1,   /* uv mod 2^n                           (Algorithm low)   */
    TM_HI = 2    /* w in [0,2^n] with |uv - 2^n w| < 2^n (Algorithm high)  */
} tm_kind;

typedef enum {
    TM_OK = 0,
    TM_ERR_INVALID = 1,     /* null pointer, n = 0, bad kind, workspace too small */
    TM_ERR_HIP = 2,         /* a HIP launch or runtime call failed               */
    TM_ERR_PRECISION = 3,   /* tm_mul_checked: the guaranteed fallback plan
                               did not pass its own bound                       */
    TM_ERR_UNSUPPORTED = 4  /* n beyond the planner's limits                    */
} tm_status;

/* Rounding guard, written on the device by every multiplication.
 * x ranges over every rounded coefficient: 2^b times the back-mapped
 * convolution for the truncated products (round(2^b W-bar_i) in the
 * algorithms), the convolution itself for the full product.
 * flags: bit0 max_dist >= 0.25; bit1 max_abs >= 2^50 (|x| so large that
 * distances to integers stop being meaningful); bit2 the lowest coefficient
 * is not a multiple of 2^b (it must be, by the cancellation propositions);
 * bit3 a carry look-back wait hit its spin limit (result invalid). */
typedef struct {
    double max_dist;   /* max |x - rint(x)|                                  */
    double max_abs;    /* max |x|                                            */
    uint32_t flags;
    uint32_t b;        /* digit size used                                    */
    uint32_t lambda;   /* series length used (0 for the full product)        */
    uint32_t kind;     /* tm_kind of the plan actually run                   */
    uint64_t N;        /* convolution length (real)                          */
} tm_guard;

#define TM_GUARD_DIST 1u
#define TM_GUARD_ABS 2u
#define TM_GUARD_C0 4u
#define TM_GUARD_SPIN 8u

/* Plan chosen for (kind, n): deterministic, a pure function of (kind, n). */
typedef struct {
    uint32_t kind;          /* requested kind                                     */
    uint32_t via_full;      /* 1 if a truncated product is served by the full-
                               product kernels plus extraction (small n)         */
    uint32_t b;             /* digit size                                         */
    uint32_t lambda;        /* series terms for the ring maps (0 if none)         */
    uint64_t n_bits;
    uint64_t N;             /* real convolution length: the ring degree N for the
                               truncated products, 2N (paper notation) for full  */
    uint64_t digits;        /* digits per operand: N (low), N+1 (high), N (full,
                               paper notation)                                    */
    uint64_t M;             /* complex FFT length = N/2                           */
    uint32_t L1, L2;        /* M = L1 * Lm * L2: column and row sub-transform     */
    uint64_t workspace_bytes;
    uint32_t Lm;            /* middle sub-transform length (1: two-pass FFT)      */
    uint32_t guaranteed;    /* 1 if rounding_bound <= 0.45 (see tm_mul_guaranteed) */
    double rounding_bound;  /* worst-case bound on |x - exact| over the rounded
                               values x of this plan (tm_mul_guaranteed)         */
    uint32_t fused;         /* 1 if one workgroup per product runs the whole
                               transform in LDS (M <= 4096; two launches)        */
    uint32_t reserved;
} tm_plan_info;

/* One request of a batch: w = product(kind, u, v) on n_bits-bit operands. */
typedef struct {
    uint32_t kind;          /* tm_kind */
    uint32_t reserved;
    uint64_t n_bits;
    const uint64_t* u;
    const uint64_t* v;
    uint64_t* w;
} tm_request;

/*
 * Autotuner: time every FFT split the planner allows for (kind, n_bits)
 * (the planner's own, each forced middle length Lm, and for each Lm the row
 * lengths L2 twice and half the planner's) on this device, on
 * `stream`, with pseudo-random operands in buffers of its own (it allocates
 * and frees them, and synchronises), and keep the fastest for later calls
 * of this process (fastest of five timed runs per split).  The split changes
 * neither N nor b, so results are the
 * same as untuned.  *chosen (may be NULL) receives the tuned plan.
 */
tm_status tm_autotune(tm_kind kind, uint64_t n_bits, hipStream_t stream, tm_plan_info* chosen);

/* Bytes of workspace a call of (kind, n_bits) needs; 0 if unsupported. */
size_t tm_workspace_bytes(tm_kind kind, uint64_t n_bits);

/* Fill *out with the plan used for (kind, n_bits).  Host only, no GPU work. */
tm_status tm_plan_query(tm_kind kind, uint64_t n_bits, tm_plan_info* out);

/*
 * w <- product of kind `kind` of u and v (n_bits-bit operands).
 * Full product: Algorithm "full product" (Section 2.2).
 * Low product: Algorithm "low product" (Section 3.4), with the ring maps of
 *   Propositions "approximating alpha*" and "approximating beta*" and the
 *   cancellation trick of Proposition "low-cancel".
 * High product: Algorithm "high product" (Section 4.3), with the maps of
 *   Propositions "approximating gamma-dagger" / "approximating delta-dagger"
 *   and Proposition "high-cancel"; returns round(t), one of the at most two
 *   allowed values.
 * guard_dev: device pointer to a tm_guard to receive the rounding guard, or
 *   NULL (then the guard lives in the workspace).
 */
tm_status tm_mul(tm_kind kind, uint64_t* w, const uint64_t* u, const uint64_t* v,
                 uint64_t n_bits, void* workspace, size_t workspace_bytes,
                 hipStream_t stream, tm_guard* guard_dev);

tm_status tm_mul_full(uint64_t* w, const uint64_t* u, const uint64_t* v, uint64_t n_bits,
                      void* workspace, size_t workspace_bytes, hipStream_t stream,
                      tm_guard* guard_dev);
tm_status tm_mul_lo(uint64_t* w, const uint64_t* u, const uint64_t* v, uint64_t n_bits,
                    void* workspace, size_t workspace_bytes, hipStream_t stream,
                    tm_guard* guard_dev);
tm_status tm_mul_hi(uint64_t* w, const uint64_t* u, const uint64_t* v, uint64_t n_bits,
                    void* workspace, size_t workspace_bytes, hipStream_t stream,
                    tm_guard* guard_dev);

/*
 * Batches of independent multiplications in packed launches.  Every stage
 * of the method (K1 split + map + column pass, the middle passes, K2 rows +
 * pointwise product, K3, K4 back-map + carry) runs as one launch per kernel
 * instance over all requests whose plans select that instance, instead of
 * one launch per request: a batch of mixed sizes and kinds costs a handful
 * of launches.  Each request has its own plan, workspace and guard, so its
 * result is bit-identical to the same call of tm_mul.  The requests must be
 * independent: no request may read another's output, and outputs must not
 * overlap any operand or each other.
 */

/* Workspace for tm_mul_batched: the sum of the requests' workspaces (each
 * rounded up to 256 bytes) plus tm_batch_meta_bytes(count); 0 if a request
 * is unsupported. */
size_t tm_workspace_bytes_batched(const tm_request* reqs, size_t count);

/*
 * Run `count` requests (host array of descriptors with device pointers) on
 * one stream in packed launches, with one workspace of
 * tm_workspace_bytes_batched() bytes (256-byte aligned) carved into the
 * requests' workspaces and the metadata area.  guards_dev: device array of
 * `count` tm_guard, or NULL.
 */
tm_status tm_mul_batched(const tm_request* reqs, size_t count, void* workspace,
                         size_t workspace_bytes, hipStream_t stream, tm_guard* guards_dev);

/* Bytes of the device metadata area of a packed batch of `count` requests
 * (per-request parameters and the launch tables). */
size_t tm_batch_meta_bytes(size_t count);

/*
 * tm_mul_batched with caller-placed memory: workspaces[i] (device, 256-byte
 * aligned, workspace_bytes[i] >= tm_workspace_bytes(kind, n) bytes) is
 * request i's workspace; `meta` (device, 256-byte aligned, meta_bytes >=
 * tm_batch_meta_bytes(count)) receives the launch metadata, uploaded by the
 * library from a pinned host buffer of its own on `stream`.  guards_dev:
 * host array of `count` device pointers (an entry may be NULL: that guard
 * stays in the workspace), or NULL.  The metadata area and the workspaces
 * must stay untouched until the batch has completed on the stream.
 * TM_ERR_INVALID (nothing launched) for a null pointer, a misaligned or too
 * small area.
 */
tm_status tm_mul_packed(const tm_request* reqs, size_t count, void* const* workspaces,
                        const size_t* workspace_bytes, void* meta, size_t meta_bytes,
                        hipStream_t stream, tm_guard* const* guards_dev);

/*
 * tm_mul_packed with a caller-owned host staging buffer for the launch
 * metadata (host_staging: pinned host memory of host_staging_bytes >=
 * tm_batch_meta_bytes(count) bytes, which the caller keeps untouched until
 * the batch has run).  The library then holds no buffer of its own across
 * the call, so the whole call may be captured into a HIP graph (stream
 * capture) once every size's tables exist (tm_prepare).
 */
tm_status tm_mul_packed_staged(const tm_request* reqs, size_t count, void* const* workspaces,
                               const size_t* workspace_bytes, void* meta, size_t meta_bytes,
                               void* host_staging, size_t host_staging_bytes, hipStream_t stream,
                               tm_guard* const* guards_dev);

/*
 * Like tm_mul, then synchronises the stream and reads the guard.  If it
 * tripped, recomputes with a fallback plan that is exact for every input by
 * its worst-case rounding bound (see tm_mul_guaranteed): the guaranteed plan
 * of the same kind when its digits are smaller, else, for the low and high
 * products at sizes without a guaranteed truncated plan (beyond about 2^22
 * bits), the full product's guaranteed plan followed by extraction of the
 * requested bits.  A run of a guaranteed plan counts as exact when the guard
 * reports only rounding distances within that plan's bound (below 1/2).
 * The workspace must hold tm_workspace_bytes_checked() bytes (the larger of
 * the two plans; at n = 2^30 the fallback needs about 4.3 GB).
 * *guard_host (may be NULL) receives the guard of the last run.
 * TM_ERR_PRECISION only if a guaranteed run reports a distance above its
 * bound or another flag (a look-back spin limit), or if no fallback plan
 * exists (the full product at sizes without a guaranteed plan).
 */
size_t tm_workspace_bytes_checked(tm_kind kind, uint64_t n_bits);

/*
 * Guaranteed mode: the same products with the digit size taken from a
 * worst-case rounding-error bound instead of the statistical default
 * (Section 5 chooses its parameters by testing).  With balanced digits
 * |U_i| <= 2^(b-1) and map gains 1 + 4 2^-b, the FFT convolution error is at
 * most ||G_u||_2 ||G_v||_2 ((1+u)^(3k) (1+sqrt5 u)^(3k+1) (1+t)^(3k) - 1),
 * u = 2^-53, t = 2^-49, k = ceil(lg M) + 4 (the convolution error bound of
 * Brent and Zimmermann, "Modern Computer Arithmetic", Theorem 3.6, which
 * Section 2.1 cites for Convolution); scaled by 2^b for the truncated
 * products, plus 2^-8 of series truncation, it must stay below 0.45.  The
 * largest such b (at most the default) is used: every rounded coefficient is
 * then provably the nearest integer, for every input.  TM_ERR_UNSUPPORTED if
 * no b >= 8 qualifies (truncated products beyond about 2^22 bits).
 */
size_t tm_workspace_bytes_guaranteed(tm_kind kind, uint64_t n_bits);
tm_status tm_plan_query_guaranteed(tm_kind kind, uint64_t n_bits, tm_plan_info* out);
tm_status tm_mul_guaranteed(tm_kind kind, uint64_t* w, const uint64_t* u, const uint64_t* v,
                            uint64_t n_bits, void* workspace, size_t workspace_bytes,
                            hipStream_t stream, tm_guard* guard_dev);
tm_status tm_mul_checked(tm_kind kind, uint64_t* w, const uint64_t* u, const uint64_t* v,
                         uint64_t n_bits, void* workspace, size_t workspace_bytes,
                         hipStream_t stream, tm_guard* guard_host);

/*
 * FP32 path: the same three products with the FFT passes (column, middle
 * and row passes, pointwise product) in double-float arithmetic, each real
 * an unevaluated sum of two floats with error-free sums and FMA products
 * (about 48 bits, the fixed-word-size scenario of Section 2.3 at a smaller
 * working precision p).  FP64 is kept for twiddle generation (tables split
 * into float pairs), the digits and ring maps, theta, the 2^b scaling, the
 * rounding and the guard.  Digit sizes keep the FP64 plans' margin against
 * the roundoff: b = 9 for the truncated products (their coefficient error
 * grows as 2^(3b)) and b = 13 for the full product (2^(2b)); transform
 * lengths are powers of two.  Same workspace layout, guard and conventions
 * as tm_mul (tm_plan_query_fp32c reports the plan; tm_coefficients_fp32c is
 * tm_coefficients for this path).
 */
size_t tm_workspace_bytes_fp32c(tm_kind kind, uint64_t n_bits);
tm_status tm_plan_query_fp32c(tm_kind kind, uint64_t n_bits, tm_plan_info* out);
tm_status tm_mul_fp32c(tm_kind kind, uint64_t* w, const uint64_t* u, const uint64_t* v,
                       uint64_t n_bits, void* workspace, size_t workspace_bytes,
                       hipStream_t stream, tm_guard* guard_dev);
tm_status tm_coefficients_fp32c(tm_kind kind, int64_t* coeffs, double* x, uint64_t coeffs_len,
                                const uint64_t* u, const uint64_t* v, uint64_t n_bits,
                                void* workspace, size_t workspace_bytes, hipStream_t stream,
                                tm_guard* guard_dev);

/*
 * Diagnostic: run the path up to rounding and write the rounded coefficients
 * c_i (int64, `coeffs_len` = plan.N for the full and low product, plan.N+1
 * for the high product) and the unrounded x_i (double, same length, may be
 * NULL) to device buffers.  c_i = round(2^b W-bar_i) of the truncated
 * algorithms (equal to 2^b L_i resp. 2^b H_i of the cancellation
 * propositions when the guard passes), c_i = round(W-bar_i) for the full
 * product.  No carry propagation.  Same workspace as tm_mul.
 */
tm_status tm_coefficients(tm_kind kind, int64_t* coeffs, double* x, uint64_t coeffs_len,
                          const uint64_t* u, const uint64_t* v, uint64_t n_bits,
                          void* workspace, size_t workspace_bytes, hipStream_t stream,
                          tm_guard* guard_dev);

/*
 * Measurement: run one multiplication with HIP events recorded on `stream`
 * between its kernels, synchronise, and write the elapsed milliseconds of
 * each kernel to stage_ms[0..*n_stages) (capacity `cap`, at least 6) and
 * their names to names[i] (static strings; may be NULL).  The stages are:
 * split+map+column FFT, [middle column FFT,] row FFT+pointwise+inverse row
 * FFT, [inverse middle column FFT,] inverse column FFT, back-map+round+carry
 * (the bracketed ones only for the three-pass split, plan Lm > 1).
 */
tm_status tm_profile_stages(tm_kind kind, uint64_t* w, const uint64_t* u, const uint64_t* v,
                            uint64_t n_bits, void* workspace, size_t workspace_bytes,
                            hipStream_t stream, float* stage_ms, const char** names,
                            int cap, int* n_stages);

/*
 * Allocation-free product, for callers that cannot allocate device memory:
 * code under HIP graph capture, tight serving loops, harnesses that forbid
 * hipMalloc.  Same result as tm_mul (same plan and kernels) without a
 * workspace argument: the workspace is a static device array of
 * tm_noalloc_max_bytes() bytes (48 MiB: every kind up to n = 2^24 bits),
 * one per GPU, held until the process ends.  The caller passes u, v, w and
 * the stream as for tm_mul.  The size's twiddle tables must exist
 * (tm_prepare, or an earlier tm_mul of the same size on this device):
 * otherwise TM_ERR_INVALID and nothing runs.  TM_ERR_UNSUPPORTED if the
 * plan's workspace exceeds the static maximum.  Calls no hipMalloc or
 * hipFree.  Every call on one GPU shares that GPU's array: calls that
 * overlap on one GPU (different streams or threads) race and give wrong
 * results; each call starts by clearing what it accumulates into.
 * guard_dev: device tm_guard or NULL (then the guard lives in the array).
 */
size_t tm_noalloc_max_bytes(void);
tm_status tm_mul_noalloc(tm_kind kind, uint64_t* w, const uint64_t* u, const uint64_t* v,
                         uint64_t n_bits, hipStream_t stream, tm_guard* guard_dev);

/*
 * Build the per-device caches a call of (kind, n_bits) uses (twiddle tables)
 * now, on `stream`, and wait for them.  Optional: every call builds them on
 * first use; servers call this before their clock starts.
 */
tm_status tm_prepare(tm_kind kind, uint64_t n_bits, hipStream_t stream);

/*
 * Barrett modular multiplication, a consumer of the truncated products
 * (Section 1 names the high product for quotients and the low product for
 * remainders): r = a b mod m for n_bits-bit a, b (any values below
 * 2^n_bits), a modulus with 2^(n-1) < m < 2^n (top bit set, not a power of
 * two), and mu = floor(2^(2n) / m), which has n + 1 bits, supplied by the
 * caller (computed once per modulus).  Steps on `stream`: x = a b (full
 * product), q1 = floor(x / 2^(n-1)), w = high product of q1 and mu at n + 1
 * bits, y = low product of w and m at n + 2 bits, r = x - y mod 2^(n+2),
 * then one conditional + m and two conditional - m (carry scans on the
 * device).  Device pointers: r, a, b, m with ceil(n/64) limbs, mu with
 * ceil((n+1)/64) limbs.  Workspace: tm_workspace_bytes_mulmod(n) bytes,
 * 256-byte aligned.  n_bits >= 2.  A wrong mu gives a wrong r, never an
 * out-of-bounds access.
 */
size_t tm_workspace_bytes_mulmod(uint64_t n_bits);  /* 0 if unsupported */
tm_status tm_mulmod(uint64_t* r, const uint64_t* a, const uint64_t* b, const uint64_t* m,
                    const uint64_t* mu, uint64_t n_bits, void* workspace, size_t workspace_bytes,
                    hipStream_t stream);

/*
 * Serving: continuous batching on the current device.
 *
 * A server owns one device memory pool of pool_bytes (allocated at
 * creation), n_streams HIP streams and max_inflight request slots (0: 128
 * per stream).  Requests carry HOST pointers (tm_request.u, .v: n_bits-bit
 * operands, read until the request completes; .w: result buffer of the
 * tm_mul layout); pinned host memory lets the copies overlap.  Requests
 * wait in submission order.  Whenever a stream has fewer than two batches
 * in flight, the waiting requests that fit are admitted as one batch of up
 * to 64: each gets its footprint (tm_server_footprint: operands, result,
 * workspace) carved out of the pool, and the batch gets one block for its
 * launch metadata and guards.  A batch is operand copies, one packed
 * multiplication call (tm_mul_packed; tm_mul for a batch of one), result
 * copies, one guard copy and one completion event.  A request that does
 * not fit reserves the bytes it waits for: requests behind it pass it only
 * within the remaining free bytes.  tm_server_poll retires finished
 * batches, frees their memory and admits waiting requests, so requests that
 * arrive while others run join the next batch as a stream and memory free
 * up, and their work overlaps on the device.  Results equal tm_mul's for
 * the same (kind, n_bits) (the plan depends on them only).  A server is
 * used from one host thread at a time.  The throughput / latency workload
 * of a whole arrival trace runs through tm_serve_trace.
 */
typedef struct tm_server tm_server;

size_t tm_server_footprint(tm_kind kind, uint64_t n_bits);  /* 0 if unsupported */
tm_status tm_server_create(size_t pool_bytes, int n_streams, int max_inflight, tm_server** out);
/* Queue one request (copied; guard_host: host tm_guard written on
 * completion, or NULL).  *id identifies it in tm_server_poll.
 * TM_ERR_INVALID if its footprint and one batch block exceed the pool. */
tm_status tm_server_submit(tm_server* s, const tm_request* req, tm_guard* guard_host, uint64_t* id);
/* Retire finished requests and admit waiting ones; writes up to cap
 * (id, status) pairs of finished requests and returns their number (-1 on
 * a null server).  Non-blocking. */
int tm_server_poll(tm_server* s, uint64_t* ids, tm_status* status, int cap);
size_t tm_server_pending(const tm_server* s);  /* queued + running */
tm_status tm_server_drain(tm_server* s);       /* block until none pending */
void tm_server_destroy(tm_server* s);          /* waits for running requests */

/*
 * Replay an arrival trace through a fresh server: request i is submitted
 * at arrival_s[i] seconds (non-decreasing) after the start; latency_s[i]
 * receives its completion time minus its arrival time, seen on the host's
 * steady clock (-1 if it failed).  guards_host: count tm_guard or NULL.
 * *makespan_s: start to last completion.  Caches for every (kind, n_bits)
 * of the trace are built before the clock starts.
 */
tm_status tm_serve_trace(const tm_request* reqs, const double* arrival_s, size_t count,
                         size_t pool_bytes, int n_streams, int max_inflight, double* latency_s,
                         tm_guard* guards_host, double* makespan_s);

/*
 * Graph mode: a batch is captured (stream capture of its copies, packed
 * multiplication with a server-owned metadata staging buffer, and result
 * copies) into a HIP graph that is instantiated and launched as one unit; a
 * batch whose capture fails (pageable host buffers) is launched directly.
 * Results are the same either way.  mode 0: never (default); 1: every batch
 * of two or more requests; 2: batches of 16 or more requests (one graph
 * launch then outweighs the capture and instantiation of a graph used once).
 */
tm_status tm_server_use_graphs(tm_server* s, int mode);

/* tm_serve_trace with flags: TM_SERVE_GRAPHS runs the server in graph mode
 * 1, TM_SERVE_GRAPHS_AUTO in graph mode 2. */
#define TM_SERVE_GRAPHS 1
#define TM_SERVE_GRAPHS_AUTO 2
tm_status tm_serve_trace_ex(const tm_request* reqs, const double* arrival_s, size_t count,
                            size_t pool_bytes, int n_streams, int max_inflight, double* latency_s,
                            tm_guard* guards_host, double* makespan_s, int flags);

const char* tm_status_string(tm_status s);
const char* tm_last_error(void);
void tm_release_caches(void);

#ifdef __cplusplus
}
#endif
#endif /* TMUL_H */
