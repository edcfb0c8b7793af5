/*
 * bqs.h -- C ABI of a BlockQuicksort-style sort for AMD Instinct MI355X
 * (gfx950).
 *
 * Operation (Edelkamp & Weiss, "BlockQuicksort: How Branch Mispredictions
 * don't affect Quicksort", arXiv 1604.06697, Introduction and Section 2):
 * rearrange a sequence of elements of a totally ordered universe into
 * ascending order, in place from the caller's point of view.  The library
 * runs Quicksort whose partitioning step is the paper's block partition
 * (Section 3, Algorithm 3) re-organised for a GPU: keys are compared with
 * the pivot a tile at a time, the comparison outcomes become offsets, and a
 * second pass moves the elements without comparison-dependent branches.
 *
 * Conventions shared by every entry point
 *   - Pointers named keys / vals / offsets / workspace are DEVICE pointers
 *     owned by the caller.  The library never allocates or frees device
 *     memory; it only owns host-side state inside a context.
 *   - Calls enqueue work on the context's HIP stream (default: the null
 *     stream) and return without waiting for it (default mode,
 *     BQS_MODE_ASYNC; BQS_MODE_LEVELS instead waits between recursion
 *     levels and returns when the sort is done).  Results are valid once
 *     the stream has passed the call, as for any kernel on that stream; the
 *     caller keeps keys, payloads, offsets and the workspace alive and
 *     unmodified until then.
 *   - Argument errors are reported at once and nothing is enqueued.
 *     Device-detected errors (a work list overflowing its capacity, a
 *     malformed offsets array, a NaN key in check mode, a device-side wait
 *     that gave up) are latched in the context when the call has completed
 *     and are returned by bqs_ctx_sync_status(); in BQS_MODE_LEVELS the
 *     call itself returns them instead.  Once a kernel has latched such an
 *     error, the call's later kernels do nothing: the keys (and payloads)
 *     are then in an unspecified state, except after malformed offsets or
 *     a NaN found by check mode, which are detected before anything moves
 *     and leave them as they were.
 *   - Keys are 1-D and contiguous.  Integer keys use their usual order;
 *     float keys use IEEE-754 totalOrder restricted to non-NaN values, so
 *     -0.0 sorts before +0.0.  NaN keys violate the precondition (their
 *     position is unspecified).
 *   - The result is unique for keys.  For key-value pairs the payload
 *     travels with its key; the order of payloads among equal keys is not
 *     specified (Quicksort is unstable, Introduction) but is deterministic
 *     for identical inputs and parameters.
 */
#ifndef BQS_H
#define BQS_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
    BQS_I32 = 1,
    BQS_U32 = 2,
    BQS_I64 = 3,
    BQS_U64 = 4,
    BQS_F32 = 5,
    BQS_F64 = 6,
    /* Not dtypes: these two widen the enum's range to every int, so an
       out-of-range value from a caller is a defined value that the library
       rejects with BQS_EDTYPE. */
    BQS_DTYPE_RANGE_MIN_ = -0x7fffffff - 1,
    BQS_DTYPE_RANGE_MAX_ = 0x7fffffff
} bqs_dtype;

typedef enum {
    BQS_OK = 0,
    BQS_EINVAL = 1,     /* bad argument: null pointer, negative size, workspace too small, ... */
    BQS_EDTYPE = 2,     /* unsupported key dtype or payload width                          */
    BQS_ENOMEM = 3,     /* host-side allocation inside the context failed                  */
    BQS_EHIP = 4,       /* a HIP runtime call failed                                        */
    BQS_ENAN = 5,       /* a floating-point key is NaN (only with BQS_PARAM_CHECK_NAN = 1)   */
    BQS_EOVERFLOW = 6,  /* a device work list or the level cap was exceeded                 */
    BQS_ETOOBIG = 7,    /* bqs_sort_noalloc: the input needs more than its fixed scratch    */
    /* Not statuses: they widen the enum's range to every int (see bqs_dtype). */
    BQS_STATUS_RANGE_MIN_ = -0x7fffffff - 1,
    BQS_STATUS_RANGE_MAX_ = 0x7fffffff
} bqs_status;

/* Tunable parameters (bqs_ctx_set_param).  Values <= 0 restore defaults. */
typedef enum {
    BQS_PARAM_SMALL_CUTOFF = 1, /* segments of at most this many keys are sorted inside one
                                   workgroup's LDS (clamped to the compiled maximum: 8192 for
                                   4-byte keys, 4096 for 8-byte keys, 2048 for pairs, which are
                                   also the defaults)                                          */
    BQS_PARAM_SAMPLE_MAX = 2,   /* largest pivot sample (<= 255; default 127, 255 with
                                   BQS_PARAM_MULTIWAY); the pivot is the median of the sample
                                   (Section 2, pivot selection)                                */
    BQS_PARAM_PIVOT_MODE = 3,   /* pivot strategy (Section 2; Section 4, pivot selection):
                                   0  median of a stratified sample of about sqrt(m)/4 keys
                                      (7 .. BQS_PARAM_SAMPLE_MAX; default);
                                   1  median of sqrt(m) keys (at most BQS_PARAM_SAMPLE_MAX),
                                      median of five medians of five below 20000 keys;
                                   3  median of the first, middle and last key;
                                   5, 23  median of 5 / 23 stratified keys;
                                   33, 35, 55  median of three medians of three, of three
                                      medians of five, of five medians of five.
                                   Past the depth limit 2 log2 n + 3 every strategy takes the
                                   largest sample.  Other values: BQS_EINVAL                    */
    BQS_PARAM_TIMING = 4,       /* HIP-event timing on the context's stream: 1 every launch
                                   (partition_ms: the partition kernels alone; plan_ms: pivots,
                                   fills, tile map and segment completion; small_ms); 2 the
                                   partition kernels only (two events per level, so the timing
                                   itself costs the host less); 0 none                          */
    BQS_PARAM_TILE_EPT = 5,     /* keys per thread in a partition tile (8, 16 or 32; 0 = auto)  */
    BQS_PARAM_GRID = 6,         /* workgroups of the persistent kernel (0 = all that can be
                                   resident at once)                                            */
    BQS_PARAM_PROFILE = 7,      /* 1: count cycles and look-back rounds inside partition tiles */
    BQS_PARAM_MODE = 8,         /* BQS_MODE_ASYNC (default), BQS_MODE_LEVELS or
                                   BQS_MODE_PERSISTENT                                          */
    BQS_PARAM_GRAPH = 9,        /* 1: capture the launches of a call into a HIP graph and replay
                                   it for later calls with the same buffers, sizes and parameters
                                   (BQS_MODE_ASYNC only; see "Graph mode" below)               */
    BQS_PARAM_ENQUEUE_LEVELS = 14, /* BQS_MODE_ASYNC: recursion levels a call enqueues before its
                                   single-workgroup tail launch (0, the default: as many as the
                                   last completed call of the same shape needed plus one, or an
                                   estimate).  The result is the same for any value; small
                                   values leave more of the recursion to the tail              */
    BQS_PARAM_DEPTH_LIMIT = 15, /* recursion depth past which every pivot is the median of the
                                   largest sample (0: the paper's 2 floor(log2 n) + 3, Section 2);
                                   the level cap is 4 times this plus 64                        */
    BQS_PARAM_LIST_CAP = 16,    /* stress test: at most this many entries in each per-level work
                                   list (segments, small segments, equal runs; 0: sized for n).
                                   A recursion that needs more latches BQS_EOVERFLOW; nothing is
                                   written past a list                                          */
    BQS_PARAM_SHUFFLE = 17,     /* stress test of the decoupled look-back (BQS_MODE_ASYNC and
                                   BQS_MODE_LEVELS): partition tiles take their tiles in reverse
                                   order within each window of 64 tickets and pause a
                                   pseudo-random time before publishing their status.  Results
                                   are identical                                                */
    BQS_PARAM_CHECK_NAN = 13,   /* 1: float keys are checked for NaN (one extra read of the keys)
                                   before the sort; a NaN is reported as BQS_ENAN and the keys
                                   are left as they were.  The sort's precondition
                                   (a totally ordered key set, Introduction) excludes NaN; 0
                                   (default) does not check                                     */
    BQS_PARAM_LOOKBACK = 10,    /* how a partition tile claims its output ranges.  0 (default):
                                   keys-only sorts move the segment's two cursors with one atomic
                                   add per tile (the paper's cursors l and r, Algorithm 3), so
                                   runs land in claim order; pairs always use the decoupled
                                   look-back.  1: every tile uses the look-back, runs land in
                                   tile order and the intermediate layout is the same on every
                                   run.  Sorted output is identical either way.                 */
    BQS_PARAM_PIVOT_SKEW = 12,  /* skewed pivots (Section 4, skewed pivot experiments): s >= 2
                                   takes the sample key of rank floor(k/s) instead of the median
                                   (s = 2 is the median; single-sample strategies only, at most
                                   64; past the depth limit the median again).  0 (default):
                                   the median.  Sorted output is identical; only the number of
                                   levels changes                                               */
    BQS_PARAM_MULTIWAY = 11,    /* 1: keys-only sorts split each segment around up to 15
                                   splitters per pass instead of one pivot (a sample-sort step:
                                   the paper's multi-pivot outlook, Section 5; 31 buckets, keys
                                   equal to a splitter finish at once), so far fewer passes
                                   run; pairs keep the two-way step.  0 (default): the paper's
                                   block partition around one pivot.  Sorted output is
                                   identical either way.                                        */
    BQS_PARAM_INPLACE = 18      /* 1: in-place levels (Section 3, Algorithm 3: the partition
                                   swaps misplaced elements inside the array instead of copying
                                   it; Section 3.2): keys and payloads never leave the caller's
                                   buffers, and the workspace holds one bit per key plus lists
                                   and per-tile counts (5 to 9 % of the default workspace;
                                   bqs_workspace_bytes reflects the setting).  Each
                                   level reads the keys twice and writes the misplaced ones once,
                                   about 1.5x the traffic of the default level.  Applies to
                                   bqs_sort, bqs_sort_pairs, bqs_sort_segments and
                                   bqs_sort_records; takes precedence over BQS_PARAM_MULTIWAY;
                                   not available in BQS_MODE_PERSISTENT (BQS_EINVAL).  Sorted
                                   keys are identical; payloads of equal keys may come out in
                                   another (still deterministic) order.  0 (default): out of
                                   place                                                        */
} bqs_param;

/* Execution modes (BQS_PARAM_MODE).
 *   ASYNC     : (default) a call enqueues every launch of the sort and
 *               returns.  Each recursion level is one partition launch whose
 *               grid covers the most tiles the level can hold; the kernels
 *               read the level's actual counts on the device.  The call
 *               enqueues as many levels as the last call of the same shape
 *               needed (plus one), or an estimate for a new shape, then one
 *               single-workgroup launch that finishes any recursion left
 *               over, so every input is sorted whatever its depth.  The
 *               context's statistics and latched status are updated when
 *               the call has completed on the device.
 *   LEVELS    : host-driven: the host reads the next level's size between
 *               levels and sizes every launch exactly; the call returns when
 *               the sort is done, with its status.
 *   PERSISTENT: every level in one cooperative launch (Quicksort's main
 *               loop, Algorithm 1, run on the device): the workgroups that
 *               fit on the GPU at once drain each level's device-resident
 *               lists -- pivots, equal runs and small segments, tile
 *               descriptors, partition tiles, segment completion -- with a
 *               grid-wide barrier between steps, and the loop ends on the
 *               device when no segment is left to partition.  Asynchronous
 *               like ASYNC.  The small-sort cutoff is clamped to 4096
 *               keys.  BQS_PARAM_GRAPH does not apply (one launch already);
 *               BQS_PARAM_MULTIWAY = 1 returns BQS_EINVAL; per-level
 *               statistics are not kept.  A barrier that waits more than
 *               about a second (the GPU cannot hold the whole grid at once)
 *               ends the launch and BQS_EHIP is latched.  Results are
 *               identical to the other modes.  Measured side effect: once a
 *               process has made a cooperative launch, its later kernels on
 *               several streams overlap less (the serving loop's capacity
 *               dropped from 18 to 11 Gkeys/s), so a process that batches
 *               work on many streams should not mix in this mode. */
typedef enum { BQS_MODE_ASYNC = 0, BQS_MODE_LEVELS = 1, BQS_MODE_PERSISTENT = 2 } bqs_mode;

/* Graph mode (BQS_PARAM_GRAPH = 1, BQS_MODE_ASYNC).  The first call with a
 * given set of buffers (keys, vals, offsets, workspace), sizes and
 * parameters captures the call's launch sequence into a HIP graph held by
 * the context and launches it; later calls with the same set replay it with
 * one hipGraphLaunch.  When a completed call shows that the shape needs a
 * different depth than the graph holds, the next call captures it again.
 * Results are identical to the default mode.  The graph reads the buffers'
 * contents at replay time, so callers refill the same buffers between
 * calls.  Kernel timings are not kept for replayed calls.  Changing any
 * parameter drops the graph.  The graph is recorded on a stream the context
 * owns (default priority) and replayed on the context's stream. */

typedef struct {
    int64_t levels;             /* levels that partitioned at least one segment               */
    int64_t partitioned_keys;   /* sum of segment sizes over all partition passes              */
    int64_t small_sorted_keys;  /* keys finished by the in-LDS small sort                       */
    int64_t filled_keys;        /* keys equal to a pivot, written by the fill step             */
    int64_t tiles;              /* partition tiles processed                                    */
    double partition_ms;        /* summed partition-kernel time (BQS_PARAM_TIMING only)         */
    int64_t partition_launches; /* partition launches enqueued (levels, plus spare levels)     */
    double small_ms;            /* summed small-sort kernel time (BQS_PARAM_TIMING = 1 only)    */
    int64_t small_launches;
    double plan_ms;             /* summed pivot, fill, map and completion kernel time          
                                   (BQS_PARAM_TIMING = 1 only)                                  */
    int64_t tile_keys;          /* compiled tile size used (keys per tile)                      */
    int64_t small_cutoff;       /* small-sort cutoff used                                       */
    /* BQS_PARAM_PROFILE only (sums over all partition tiles; cycles of the shader clock): */
    int64_t prof_tiles;
    int64_t prof_lookback_rounds;   /* 64-tile windows read by look-backs                          */
    int64_t prof_lookback_polls;    /* status reads including re-polls of unpublished tiles        */
    double prof_lookback_cycles;    /* wave 0 time from its scan result to the claimed range       */
    double prof_tile_cycles;        /* tile start to tile end                                      */
    double prof_load_cycles;        /* tile start to all keys loaded and counted                   */
    int64_t graph_launches;         /* 1 if the call replayed a captured graph                     */
    /* BQS_PARAM_PROFILE only: small segments sorted, and the shader-clock cycles of each phase of
       the small sort, summed over segments: key load and range, bucket counts, bucket starts,
       scatter into buckets, order inside buckets and store */
    int64_t prof_small_segments;
    double prof_small_cycles[5];
} bqs_stats;

typedef struct bqs_ctx bqs_ctx; /* opaque, host-side */

/* Creates a context.  Host memory only; no GPU call is made.  *out receives
 * the handle; returns BQS_EINVAL if out is NULL, BQS_ENOMEM on failure. */
bqs_status bqs_ctx_create(bqs_ctx** out);

/* Destroys a context (NULL is allowed).  Does not touch caller memory. */
void bqs_ctx_destroy(bqs_ctx* ctx);

/* Sets the HIP stream (a hipStream_t passed as void*) on which all work of
 * this context is enqueued.  NULL selects the null stream. */
bqs_status bqs_ctx_set_stream(bqs_ctx* ctx, void* hip_stream);

/* Hands the context a caller-owned device buffer of `bytes` bytes used as
 * scratch by the next calls (double buffer, work lists, tile status words).
 * Its size must be at least bqs_workspace_bytes() of the call.  The library
 * keeps the pointer only; the caller keeps it alive while calls run. */
bqs_status bqs_ctx_set_workspace(bqs_ctx* ctx, void* dev_ptr, size_t bytes);

bqs_status bqs_ctx_set_param(bqs_ctx* ctx, int param, int64_t value);
int64_t bqs_ctx_get_param(const bqs_ctx* ctx, int param);

/* Statistics of the most recent call on this context; waits until the
 * calls it has enqueued have completed on the device. */
bqs_status bqs_ctx_get_stats(bqs_ctx* ctx, bqs_stats* out);

/* Per-level statistics of the most recent call (waits like
 * bqs_ctx_get_stats): keys partitioned by level `level` (0-based; levels
 * past 127 are summed into level 127) and, with BQS_PARAM_TIMING, that
 * level's partition kernel time in ms.  Either output pointer may be NULL.
 * Returns BQS_EINVAL for a level the call did not run. */
bqs_status bqs_ctx_get_level(bqs_ctx* ctx, int level, int64_t* keys, double* partition_ms);

/* Workspace needed to sort n_total keys of `key` type with `val_bytes`-byte
 * payloads (0 for keys only) split into k_segments segments (1 for a single
 * array), under the context's current parameters (ctx may be NULL for the
 * defaults).  Returns 0 for an unsupported dtype / payload width. */
size_t bqs_workspace_bytes(const bqs_ctx* ctx, int64_t n_total, bqs_dtype key, int32_t val_bytes,
                           int64_t k_segments);

/* Sorts keys[0..n) ascending (Introduction: the problem statement; the
 * recursion follows Algorithm 1 with the improvements of Section 2).
 * keys: device pointer, n elements of `dtype`, 4-byte aligned (8 for 64-bit
 * keys).  n < 0 or keys == NULL with n > 0 -> BQS_EINVAL.  n <= 1 is a
 * no-op.  Each segment handled by a partition pass must hold fewer than
 * 2^31 keys. */
bqs_status bqs_sort(void* keys, int64_t n, bqs_dtype dtype, bqs_ctx* ctx);

/* Sorts (keys[i], vals[i]) records by key: the payload moves with its key
 * (the paper's records compared by a key field, Section 4, experimental
 * setup; the partition moves whole elements, Algorithm 3).  vals: device
 * pointer to n payloads of val_bytes (4 or 8) bytes each; keys and vals
 * must not overlap each other or the workspace.  Errors as for bqs_sort;
 * val_bytes other than 4 or 8 -> BQS_EDTYPE. */
bqs_status bqs_sort_pairs(void* keys, void* vals, int64_t n, bqs_dtype key, int32_t val_bytes,
                          bqs_ctx* ctx);

/* Sorts k independent segments keys[offsets[i] .. offsets[i+1]) in one
 * batched launch sequence: the problem statement (Introduction) applied to
 * each segment, the segments entering the recursion as level 0's list
 * (Algorithm 1's stack seeded with k ranges).  offsets: device pointer to
 * k+1 int64 values, offsets[0] = 0, non-decreasing, offsets[k] = n_total
 * (the caller passes n_total so no device read-back is needed to size the
 * work); each segment holds fewer than 2^31 keys.  A malformed offsets
 * array is detected on the device; nothing is sorted and BQS_EINVAL is
 * latched. */
bqs_status bqs_sort_segments(void* keys, const int64_t* offsets, int64_t k, int64_t n_total,
                             bqs_dtype dtype, bqs_ctx* ctx);

/* Segmented form of bqs_sort_pairs: each segment's (key, payload) records
 * are sorted by key, payloads moving with their keys; offsets, n_total and
 * error behaviour as for bqs_sort_segments, vals as for bqs_sort_pairs. */
bqs_status bqs_sort_segments_pairs(void* keys, void* vals, const int64_t* offsets, int64_t k,
                                   int64_t n_total, bqs_dtype key, int32_t val_bytes, bqs_ctx* ctx);

/* For callers that cannot allocate device memory -- code under HIP graph
 * capture, serving loops and harnesses that forbid allocation: bqs_sort
 * without a caller workspace or a context.  The workspace is a fixed 64 MiB
 * array in device memory owned by the library (one per GPU, held until the
 * process ends), so the call allocates nothing, on the device or through
 * any library routine, and only enqueues kernels on `hip_stream` (a
 * hipStream_t of the current device, NULL for the null stream) with the
 * library's default parameters.
 *   keys, n, dtype : as for bqs_sort (keys: device pointer, n < 2^31).
 *   status_out     : device pointer to one int32 that receives the call's
 *                    bqs_status (BQS_OK, or a device-detected error) when
 *                    the stream reaches the end of the sort; NULL: none.
 * Returns BQS_ETOOBIG, with nothing enqueued, when the sort needs more than
 * the scratch: n up to bqs_workspace_bytes(NULL, n, dtype, 0, 1) <= 64 MiB,
 * about 16.4 million 4-byte or 8.08 million 8-byte keys.  Other argument
 * errors as for bqs_sort.  Every call on a GPU shares that GPU's scratch
 * (which keeps the last call's contents; every call starts by clearing what
 * must start at zero): calls that overlap on one GPU -- on different
 * streams, or from different threads -- race and must not be made. */
bqs_status bqs_sort_noalloc(void* keys, int64_t n, bqs_dtype dtype, void* hip_stream, int32_t* status_out);

/* The paper's large element types (Section 4, experimental setup):
 *   BQS_RECORD_VECTOR: 10 doubles (80 bytes), ordered by the sum of the
 *     squares of the components (left to right, every product and sum
 *     rounded, no fused multiply-add); no NaN or infinite components;
 *   BQS_RECORD_RECORD: 21 int32 (84 bytes), ordered by the first component.
 * bqs_sort_records sorts n records from `in` into `out` (device pointers,
 * caller-owned, not overlapping each other or the workspace): it computes
 * every record's key once, sorts (key, index) pairs with bqs_sort_pairs'
 * machinery (host-driven; BQS_PARAM_GRAPH does not apply) and gathers the
 * records in key order.  Records with equal keys come out in an unspecified
 * order (Quicksort is not stable).  n >= 2^31 -> BQS_EINVAL; an unknown kind
 * -> BQS_EDTYPE.  The workspace must hold bqs_records_workspace_bytes(n,
 * kind) bytes. */
typedef enum { BQS_RECORD_VECTOR = 1, BQS_RECORD_RECORD = 2 } bqs_record;
size_t bqs_records_workspace_bytes(const bqs_ctx* ctx, int64_t n, int kind);
bqs_status bqs_sort_records(const void* in, void* out, int64_t n, int kind, bqs_ctx* ctx);

/* Waits until every call enqueued on this context has completed (and
 * synchronises the context's stream), then returns the first error latched
 * since the previous bqs_ctx_sync_status() -- a device-detected error of a
 * call, or an error an asynchronous call returned -- and clears it. */
bqs_status bqs_ctx_sync_status(bqs_ctx* ctx);

/* Completion clock of segmented calls (for callers that measure per-segment
 * latency inside one batched call).  For the bqs_sort_segments and
 * bqs_sort_segments_pairs calls made on this context from now on, `ticks`
 * (a device array of at least k + 1 entries, caller-owned, kept alive until
 * the calls complete) receives at [i] the device wall clock (a 100 MHz
 * counter) at which the last key of segment i reached its final place --
 * after the kernel that finished it had issued its stores -- and at [k]
 * the clock when the call's first kernel started.  Segments of at most one
 * key get that start time.  A call with more segments than
 * `count` - 1 fails with BQS_EINVAL; a call that does no work (k = 0 or
 * n_total <= 1) writes nothing.  ticks = NULL turns the clock off.  Changing
 * it drops a captured graph.  The clock costs one atomic per finished
 * piece. */
bqs_status bqs_ctx_set_segment_ticks(bqs_ctx* ctx, uint64_t* ticks, int64_t count);

/* Returns the first error latched by this context's calls that have
 * completed so far -- without waiting for the calls still running -- and
 * clears it (BQS_OK when there is none).  For callers that track each
 * call's completion themselves (an event recorded after the call) and
 * must not block on the calls enqueued after it. */
bqs_status bqs_ctx_poll_status(bqs_ctx* ctx);

/* Static, human-readable name of a status code. */
const char* bqs_status_str(bqs_status status);

/* Library version as MAJOR*10000 + MINOR*100 + PATCH. */
int bqs_version(void);

#ifdef __cplusplus
}
#endif

#endif /* BQS_H */
