/*
 * lsort -- LearnedSort 2.0 on one AMD Instinct MI355X (gfx950).
 *
 * C ABI of the GPU library (liblsort.so).  The method is LearnedSort 2.0
 * (Kristo, Vaidya, Kraska, arXiv 2107.03290): a two-layer linear eCDF model
 * trained on a 1% sample predicts each key's bucket (Sec. 2, Sec. 6.1),
 * keys are partitioned by those predictions (Alg. 1), buckets whose keys
 * are all equal are never partitioned again (Alg. 2, Sec. 4.2), the rest
 * are partitioned again and finally sorted inside the bucket, and a touch-up
 * pass guarantees the order (Alg. 2, last step).
 *
 * Conventions for every call:
 *  - Key buffers are DEVICE memory owned by the caller; they are sorted IN
 *    PLACE, asynchronously on the given HIP stream (NULL = default stream).
 *    A call returns once the work is enqueued, except where noted.
 *  - The library owns its scratch (about one key buffer's worth of device
 *    memory plus small tables); it grows on first use and is then reused, so
 *    repeated calls with the same or smaller sizes allocate nothing.
 *  - Every call returns an ls_status and never throws.  Argument errors are
 *    reported before any work is enqueued.  ls_last_error() describes the
 *    most recent failure of a context.
 *  - A context is not thread-safe: use one per host thread (the server
 *    below owns its own context).
 *  - Result: the unique non-decreasing permutation of the input.  u64 keys
 *    use unsigned order; f64 keys use IEEE-754 totalOrder on the bit
 *    patterns (-NaN < -inf < ... < -0.0 < +0.0 < ... < +inf < +NaN), so the
 *    output is bit-exact and independent of every tuning parameter.
 */
#ifndef LSORT_H
#define LSORT_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct ihipStream_t* ls_stream_t;   /* a hipStream_t */

typedef enum {
    LS_OK = 0,
    LS_ERR_INVALID = 1,      /* bad argument (null pointer with n > 0, bad dtype, bad offsets, bad params) */
    LS_ERR_NOMEM = 2,        /* device or host allocation failed */
    LS_ERR_HIP = 3,          /* a HIP runtime call failed */
    LS_ERR_UNSUPPORTED = 4,  /* parameter combination not supported */
    LS_ERR_BUDGET = 5,       /* server: a request larger than the whole HBM budget */
    LS_ERR_TIMEOUT = 6,      /* server: wait timed out */
    LS_ERR_NOTFOUND = 7      /* server: unknown ticket */
} ls_status;

typedef enum { LS_F64 = 1, LS_U64 = 2 } ls_dtype;

/* ls_params.flags */
#define LS_FLAG_DEBUG_TOUCHUP  0x1u   /* check every adjacent pair after the sort, not only bucket seams */
#define LS_FLAG_SYNC           0x2u   /* wait for the stream before returning */
#define LS_FLAG_NONMONOTONE    0x4u   /* test hook: perturb predictions so buckets overlap; the touch-up must repair */
#define LS_FLAG_PROFILE        0x8u   /* time each kernel class with HIP events (read with ls_last_profile) */
/* With LS_FLAG_PROFILE: time only kernel class k (0..7, the classes of
 * ls_last_profile).  Each event pair costs the stream a few microseconds at
 * a class boundary; with this bit the other classes run back to back. */
#define LS_FLAG_PROFILE_ONLY(k) (((uint32_t)(k) + 1u) << 8)
#define LS_FLAG_GRAPH          0x10u  /* run a batch of at most 2^22 keys and 2^16 arrays as one replay of a HIP
                                         graph captured for its size class (keys and arrays rounded up to powers
                                         of two); the first batch of a class captures it.  Results are the same
                                         as without the flag.  Ignored with LS_FLAG_PROFILE or
                                         LS_FLAG_DEBUG_TOUCHUP and for larger batches. */

#define LS_FLAG_INPLACE        0x20u  /* partition in place (Alg. 1: fragments of 64 keys written back into the
                                         input, then Defragment as a block permutation) instead of through a
                                         scratch buffer of n keys: extra device memory per round is about 3% of
                                         the keys' bytes.  Fanout is capped at 128.  Same results; slower. */

/* Tuning parameters (Sec. 6.1 gives f = 1000, c = 100, L = 1000, 1% sample).
 * Zero fields take the library defaults.  None of them changes the result. */
typedef struct {
    uint32_t struct_size;      /* sizeof(ls_params) */
    uint32_t fanout;           /* f: buckets per partition, 2..4096 (default 1024) */
    uint32_t leaves;           /* L: leaf models of the two-layer model, 1..1024 (default 1024) */
    uint32_t tile;             /* keys staged per scatter tile in LDS: at most 1024, 2048, 4096 or 8192
                                  (halved down to 1024 while the tile, the fanout's tables and the model
                                  exceed a workgroup's LDS), or 0 (ls_default_params) for automatic: 4096,
                                  and 8192 in host-driven rounds of at least 2^25 keys whose fanouts leave
                                  room for it in LDS; 12288 instead (32-bit cursors) in such rounds of
                                  fewer than 2^31 keys when leaves <= 512 and the fanouts fit (at most
                                  1202 with 512 leaves) */
    uint32_t base_threshold;   /* buckets of at most this many keys are sorted in LDS, in groups of < 2x (default 4096, max 4096) */
    uint32_t flags;            /* LS_FLAG_* */
    double   sample_rate;      /* model training sample (default 0.01) */
    uint64_t sample_cap;       /* upper bound on one model's sample (ls_default_params: 262144, so the
                                  1% rate holds up to 26.2M keys); 0 = none.  A NULL ls_params
                                  uses the default. */
    uint64_t seed;             /* seed of the counter-based sampler */
} ls_params;

typedef struct ls_ctx ls_ctx;

/* Device status bits returned by ls_sync. */
#define LS_DEV_SEAM_REPAIRED   0x1u   /* the touch-up found an out-of-order seam and repaired it */
#define LS_DEV_FALLBACK        0x2u   /* a bucket needed the highest-differing-bit split (no model progress) */
#define LS_DEV_DEEP            0x4u   /* recursion went deeper than two levels */

/* Create a context on HIP device `device` (the device becomes current). */
ls_status ls_create(ls_ctx** out, int device);
/* Wait for the context's queued work (not the whole device's), then free it. */
ls_status ls_destroy(ls_ctx* ctx);

/* Fill *p with the defaults. */
void ls_default_params(ls_params* p);

/* Device bytes of work buffers a sort of n keys needs (an estimate: the
 * scratch keys, or about n B in place with LS_FLAG_INPLACE, plus round
 * tables, output lists and training samples).  ctx may be NULL. */
ls_status ls_workspace_size(ls_ctx* ctx, ls_dtype dtype, size_t n, const ls_params* p, size_t* bytes);

/* Allocate scratch for sorts of up to n keys ahead of time. */
ls_status ls_reserve(ls_ctx* ctx, size_t n, const ls_params* p);

/* Device memory the context holds now, in bytes: the sum of its work buffers
 * (scratch keys, round tables, output lists, training samples), which it
 * keeps between sorts and grows on demand.  Not counted: the library's code
 * and static data, and what the HIP runtime allocates for itself.  Waits for
 * nothing; call it when no sort of this context is being issued. */
ls_status ls_device_bytes(ls_ctx* ctx, size_t* bytes);

/* Wait for the context's queued work, then free all its work buffers (the
 * next sort allocates them again).  Graphs recorded on them are dropped. */
ls_status ls_trim(ls_ctx* ctx);

/* Sort n keys of d_keys in place (Alg. 2).  d_keys: device pointer to n
 * contiguous 8-byte keys, 8-byte aligned.  p may be NULL (defaults). */
ls_status ls_sort_f64(ls_ctx* ctx, double* d_keys, size_t n, ls_stream_t stream, const ls_params* p);
ls_status ls_sort_u64(ls_ctx* ctx, uint64_t* d_keys, size_t n, ls_stream_t stream, const ls_params* p);

/* Largest n ls_sort_noalloc takes. */
#define LS_NOALLOC_MAX_KEYS (1u << 20)

/* For callers that cannot allocate memory (code that must not call
 * hipMalloc: tight serving loops, harnesses that forbid allocation, setups
 * that reserve all other device memory): the same sort as ls_sort_f64 /
 * ls_sort_u64 (dtype selects which), giving the same bits, but every device
 * buffer it needs is cut from one static 128 MiB array per device that is
 * part of the library's code object (loaded, and held until the process
 * ends, on each device the library runs on; its address is looked up by
 * ls_create).  The call allocates no device or pinned memory and grows no
 * buffer of the context.
 *  - n <= LS_NOALLOC_MAX_KEYS (1,048,576); a larger n is rejected with
 *    LS_ERR_UNSUPPORTED before any work.  Parameters whose tables do not fit
 *    the array for this n (a fanout of 4096 at the largest n, a tiny
 *    base_threshold) are rejected the same way; the defaults always fit.
 *  - LS_FLAG_PROFILE and LS_FLAG_GRAPH are rejected (LS_ERR_UNSUPPORTED).
 *  - Synchronous: returns once the sort is complete.
 *  - Every call on a device shares that device's array and leaves its
 *    contents behind; the call clears what must start at zero.  Calls that
 *    overlap on one device (other contexts, other threads) race on the array
 *    and corrupt each other's results: serialise them. */
ls_status ls_sort_noalloc(ls_ctx* ctx, ls_dtype dtype, void* d_keys, size_t n, ls_stream_t stream,
                          const ls_params* p);

/* Sort many independent arrays in one batched pipeline.  d_keys holds the
 * segments back to back; h_offsets (HOST memory, num_segments + 1 entries,
 * non-decreasing, h_offsets[0] = 0) gives each segment's key range.
 * h_dtypes (HOST, num_segments entries of ls_dtype values) may be NULL, in
 * which case every segment has type `dtype`.  Each segment ends up sorted
 * exactly as a separate ls_sort_* call would sort it. */
ls_status ls_sort_segments(ls_ctx* ctx, ls_dtype dtype, void* d_keys, const uint64_t* h_offsets,
                           size_t num_segments, const uint8_t* h_dtypes, ls_stream_t stream,
                           const ls_params* p);

/* ls_sort_segments with the batch described on the DEVICE: d_offsets
 * (num_segments + 1 entries, d_offsets[0] = 0, non-decreasing) and d_dtypes
 * (num_segments ls_dtype bytes, or NULL for `dtype`) in device memory, so a
 * batch already resident on the device needs no host copy of its
 * description.  A kernel prepares round 0 from them (groups of small
 * segments, one global-model task per large segment); the host reads back
 * only the total key count (to size the scratch) and round 0's counts.
 * Invalid offsets are found on the device and reported as LS_ERR_INVALID.
 * The same result as ls_sort_segments.  LS_FLAG_GRAPH is ignored
 * (host-driven rounds).  Returns once round 0's counts are read; the sort
 * completes on `stream`. */
ls_status ls_sort_segments_device(ls_ctx* ctx, ls_dtype dtype, void* d_keys, const uint64_t* d_offsets,
                                  size_t num_segments, const uint8_t* d_dtypes, ls_stream_t stream,
                                  const ls_params* p);

/* One array of a batch: its own device buffer, length and key type. */
typedef struct {
    void*    d_keys;
    uint64_t n;
    uint32_t dtype;            /* ls_dtype */
    uint32_t reserved;
} ls_array;

/* Sort `count` separate device arrays together (the segmented pipeline
 * without the shared buffer).  h_arrays is HOST memory. */
ls_status ls_sort_arrays(ls_ctx* ctx, const ls_array* h_arrays, size_t count, ls_stream_t stream,
                         const ls_params* p);

/* One configuration timed by ls_autotune. */
typedef struct {
    uint32_t fanout;
    uint32_t tile;
    uint32_t base_threshold;
    uint32_t reserved;
    double   ms;               /* fastest repetition; < 0: does not fit this device, not run */
} ls_tune_result;

/* LearnedSort 1.0's spill bucket, as an ablation against the fragment
 * partition (Sec. 2, Fig. 1, Sec. 3).  Sorts d_keys (device, n keys of
 * dtype, in place; the same result as ls_sort_f64/u64) the way LS1 did:
 * one partition by the global model into p->fanout buckets of fixed
 * capacity ceil(n (1 + slack) / fanout); the keys a full bucket cannot take
 * go to a spill bucket.  The buckets are sorted (this library's pipeline,
 * as segments), the spill bucket by a general-purpose sort (rocPRIM's radix
 * sort, standing in for LS1's std::sort), and the two are merged (rocPRIM).
 * With many repeated keys the spill bucket grows, and so does the work of
 * the last two steps.  out8 (host, may be NULL): [0] spilled keys, [1] the
 * capacity, [2] ms partition (model, counts, scatter), [3] ms bucket sorts,
 * [4] ms spill sort, [5] ms pack, merge and conversion, [6] ms in all,
 * [7] fanout.  Synchronous.  Device memory: about (2 + slack) n x 8 B plus
 * 2 x 8 B per spilled key, besides the sort's own scratch. */
ls_status ls_sort_ls1(ls_ctx* ctx, ls_dtype dtype, void* d_keys, size_t n, double slack, ls_stream_t stream,
                      const ls_params* p, double* out8);

/* Autotuner for the GPU-specific knobs (fanout, LDS tile, base-case
 * threshold; the paper fixes f = 1000, c = 100 for its CPU, Sec. 6.1).
 * Sorts a library-owned copy of the `count` arrays (HOST list, device keys;
 * the caller's keys are NOT modified) once per candidate and repetition,
 * timed with HIP events on `stream`, and writes the fastest configuration to
 * *best (every other field copied from `base`, which may be NULL).  The
 * candidates are fanout in {512, 1024, 2048, 4096} x tile in {2048, 0 (automatic)} x
 * base_threshold in {1024, 2048, 4096}.  No candidate changes the sorted
 * result, so tuning only affects speed.  results (HOST, may be NULL) receives
 * up to cap entries and *n_results the number of candidates.  reps = 0 means
 * 2.  Synchronous; needs device memory for one more copy of the keys. */
ls_status ls_autotune(ls_ctx* ctx, const ls_array* h_arrays, size_t count, ls_stream_t stream,
                      const ls_params* base, uint32_t reps, ls_params* best, ls_tune_result* results,
                      size_t cap, size_t* n_results);

/* Wait for the context's last sort (its queued work only) and report device
 * status bits (LS_DEV_*); device_status may be NULL. */
ls_status ls_sync(ls_ctx* ctx, uint32_t* device_status);

/* Counters of the last completed sort (filled by ls_sync):
 * [0] partition rounds, [1] tasks partitioned, [2] LDS base-case groups,
 * [3] all-equal buckets filled without sorting, [4] keys in those buckets,
 * [5] fallback splits, [6] out-of-order seams repaired, [7] deepest level. */
ls_status ls_last_stats(ls_ctx* ctx, uint64_t* out8);

/* Per kernel class, accumulated since the last ls_profile_reset (only for
 * sorts run with LS_FLAG_PROFILE): out[3*k + 0] milliseconds, [3*k + 1]
 * launches, [3*k + 2] algorithmic bytes (keys read + written as the method
 * requires: the histogram reads each key of a round once, the scatter reads
 * each key of a progressing range and writes each one outside all-equal
 * buckets; both evaluate each key's bucket from the model, nothing is
 * stored in between).  Classes k: 0 train, 1 histogram, 2 scan, 3 classify,
 * 4 scatter, 5 base case, 6 fill, 7 touch-up.  cap >= 24. */
ls_status ls_last_profile(ls_ctx* ctx, double* out, size_t cap);
ls_status ls_profile_reset(ls_ctx* ctx);

const char* ls_status_string(ls_status s);
const char* ls_last_error(ls_ctx* ctx);

/* ---- stage hooks for parity checks against a reference implementation ---- */

/* Train the global model on the sample of d_keys[0..n) (Sec. 6.1: a 1%
 * sample, two layers) and copy it to h_model_out (HOST, cap doubles) in the
 * layout [xmin, xmax, rs, m'] + for each of the L leaf knots and then the
 * start knot (at the sample minimum) [X, y, ym, y1, ylo, yhi, s]: the knot,
 * the sample eCDF below it, at it (mid-rank) and at-or-below it, and the
 * segment above it (from ylo with slope s, up to yhi); a leaf with no sample
 * value has X = +inf.  4 + 7 (L + 1) doubles.  Synchronous. */
ls_status ls_model_train(ls_ctx* ctx, ls_dtype dtype, const void* d_keys, size_t n,
                         const ls_params* p, double* h_model_out, size_t cap);

/* One partition histogram (Alg. 1 bucket sizes S_B plus per-bucket
 * min/max of the order-preserving key words) of d_keys[0..n) with a model
 * given in the layout above (HOST, `leaves` leaves): bucket of x is
 * clamp(floor(F(x) * scale) - offset, 0, fanout - 1).  Outputs are HOST
 * arrays of `fanout` entries; empty buckets report min = ~0, max = 0.
 * Synchronous. */
ls_status ls_stage_hist(ls_ctx* ctx, ls_dtype dtype, const void* d_keys, size_t n,
                        const double* h_model, uint32_t leaves, double scale, int64_t offset,
                        uint32_t fanout, uint64_t* h_counts, uint64_t* h_min, uint64_t* h_max);

/* ---- serving: continuous batching of sort requests ---- */

typedef struct ls_server ls_server;

/* Start a server on `device` with max_inflight workers, each with its own
 * context and stream, so that up to max_inflight batches run on the device
 * at once.  A free worker batches queued requests into one segmented sort.
 * Admission keeps the accounted device memory within hbm_budget_bytes:
 * the keys of the requests being sorted (n x 8 B each, the caller's
 * buffers), plus every worker's context.  An idle context counts what it
 * holds (ls_device_bytes).  A busy one counts that plus a bound on what its
 * batch can add (1.5 x ls_workspace_size, since a buffer grows by at least
 * half of itself).  A worker whose own retained buffers keep the oldest
 * request out frees them (ls_trim) first.  p may be NULL (the defaults);
 * with LS_FLAG_INPLACE the batches need about n B instead of n x 8 B of
 * scratch.  With LS_FLAG_GRAPH, batches of at most 2^22 keys run as replays
 * of graphs that each worker captures per size class. */
ls_status ls_server_create(ls_server** out, int device, size_t hbm_budget_bytes,
                           uint32_t max_inflight, const ls_params* p);

/* Queue a request: sort d_keys (device, n keys of dtype) in place.  Returns
 * immediately with a ticket.  A request that can never fit the budget (its
 * keys and its batch bound alone exceed it) is rejected with LS_ERR_BUDGET;
 * one that fits later waits in the queue. */
ls_status ls_server_submit(ls_server* s, ls_dtype dtype, void* d_keys, size_t n, uint64_t* ticket);

/* Wait for a ticket (timeout_ms < 0: forever).  latency_s receives the time
 * from submission to completion on the device clock of the host. */
ls_status ls_server_wait(ls_server* s, uint64_t ticket, int timeout_ms, double* latency_s);

/* Server counters: [0] submitted, [1] completed, [2] batches, [3] peak
 * accounted bytes, [4] accounted bytes now (keys being sorted + what the
 * workers' contexts hold or have reserved), [5] queued requests. */
ls_status ls_server_stats(ls_server* s, uint64_t* out6);

/* Copy the message of the latest failed batch (empty if none) into buf
 * (cap bytes, NUL-terminated, truncated to fit). */
ls_status ls_server_last_error(ls_server* s, char* buf, size_t cap);

/* Drain every request and stop. */
ls_status ls_server_destroy(ls_server* s);

#ifdef __cplusplus
}
#endif
#endif
