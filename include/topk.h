/*
 * libtopk — unsorted top-k selection on one AMD Instinct MI355X (gfx950).
 *
 * Method: the sampling selection of Hübschle-Schneider, Sanders, Müller,
 * "Communication Efficient Algorithms for Top-k Selection Problems":
 * §2 (Algorithm "communication efficient selection": pick two pivots from a
 * sorted random sample, three-way partition, recurse into the part that holds
 * rank k) with §4.1's Bernoulli sampling of the current subproblem.
 *
 * Problem (§4): identify the elements of rank <= k among n keys.  The order is
 * made unique by pairing each value with its object (§2, Preliminaries); the
 * object is the 0-based position of the key (the row-local position in the
 * batched and row-wise calls), so ties are broken by ascending position.
 *   - u32 keys: unsigned order.
 *   - f32 keys: IEEE order with -0.0 == +0.0; every NaN (any sign, any
 *     payload) equals every other NaN and is above +inf.
 *   - TOPK_LARGEST reverses the value order; ties still go by ascending
 *     position.
 * The result is exact and does not depend on the random sample, which only
 * steers the running time.
 *
 * Conventions for every call below
 *   - Pointers are device pointers (hipMalloc / torch CUDA tensors) unless
 *     marked "host".  `keys` is never written.  Outputs and the workspace are
 *     owned by the caller.  No call allocates device memory.
 *   - Calls are asynchronous on `stream`: results are valid once the stream
 *     reaches the call.  Argument errors are reported synchronously by the
 *     return value and then nothing is enqueued.  Errors found while the
 *     kernels run are reported in the device `status` word.
 *   - Keys must be 4-byte aligned; any 4-byte alignment is accepted.
 *   - A context holds host state only (parameters, seed).  Use one context
 *     per host thread at a time.  Calls that share a workspace must be
 *     ordered on one stream.
 *   - No C++ exception crosses this interface.
 */
#ifndef TOPK_H
#define TOPK_H

#include <stddef.h>
#include <stdint.h>
#include <hip/hip_runtime_api.h>

#ifdef __cplusplus
extern "C" {
#endif

/* Return codes. */
#define TOPK_OK 0
#define TOPK_E_INVALID (-1)      /* null pointer, n or k out of range, bad flag/param */
#define TOPK_E_WORKSPACE (-2)    /* ws_bytes smaller than the *_workspace_bytes figure */
#define TOPK_E_HIP (-3)          /* a HIP runtime call or kernel launch failed */
#define TOPK_E_UNSUPPORTED (-4)  /* device is not gfx950 */

/* Flags. */
#define TOPK_LARGEST 1u          /* select the k largest instead of the k smallest  */
#define TOPK_SORTED 2u           /* single selection: out_idx in (key, position) order */
#define TOPK_WRITE_KEYS 4u       /* also write the selected keys (original bits)   */
#define TOPK_TRACE 8u            /* record every round's sample in the workspace   */
#define TOPK_GRAPH 16u           /* batched: launch through a cached hipGraph      */

/* Device status word bits (written by every select call when status != NULL). */
#define TOPK_STATUS_OK 0u
#define TOPK_STATUS_INTERNAL 1u        /* an internal consistency check failed (a
                                          library defect); outputs invalid          */
#define TOPK_STATUS_BAD_ROW 2u         /* batched: some row had k = 0 or k > len      */
#define TOPK_STATUS_BAD_KEY 4u         /* frequent / sum: a key >= U was skipped      */
#define TOPK_STATUS_SUM_RANGE 8u       /* sum: the sum of all values is >= 2^63, so
                                          the weighted sample is empty              */
#define TOPK_STATUS_BAD_ARG 16u        /* sorted rows: k (or kmin) outside [1, n], or
                                          positions beyond 32 bits; nothing written */

typedef struct topk_ctx topk_ctx;

/* Create a context on HIP device `hip_device` (must be gfx950).  `seed` keys
 * the counter-based random stream (Philox4x32-10) of the sampler.  The
 * selected set, the k-th key and its position never depend on the seed or on
 * any parameter; only the running time and the round trace do.
 * Returns TOPK_OK and *out, TOPK_E_INVALID (out NULL), TOPK_E_HIP or
 * TOPK_E_UNSUPPORTED. */
int topk_create(topk_ctx **out, int hip_device, uint64_t seed);
void topk_destroy(topk_ctx *ctx);

/* Tuning parameters (host).  Names and defaults:
 *   "s_target"   4096  expected sample size per round (§4.1 samples the
 *                      current subproblem at rate s_target / n_cur); 16..8192
 *   "c_num"      16    pivot spread c = c_num / 4; the pivots are the sample
 *                      elements of rank k s/n -/+ Delta, Delta = ceil(c sqrt(
 *                      m_hi (s - m_lo) / s)) + 1 (§2, FR-selection); 0..4096
 *   "t_fin"     16384  subproblems of at most this size are solved directly
 *                      in one workgroup (§2 base case); 1..16384
 *   "r_max"      24    sampling attempts (rounds + repeated rounds); 1..32.
 *                      Once spent, the object of rank k of the remaining
 *                      subproblem is found exactly by a streaming radix select
 *                      (one workgroup) and the call finishes with it: every
 *                      valid call terminates with the exact result
 *   "r_fast"     -1    multi-workgroup rounds enqueued before the single-
 *                      workgroup tail; -1 = chosen from n and k; 0..8
 *   "band_div"   4     the middle part b of a round may hold n/band_div + 65536
 *                      elements before the round is repeated; 1..64
 *   "tail_max"   65536 the host's round estimate stops enqueueing multi-
 *                      workgroup rounds once the expected middle part is below this
 *   "timing"     0     1: record HIP events around each call's first sweep
 *                      kernel; 2: around every kernel (see topk_kernel_times)
 *   "seed"             the sampler seed (also set by topk_create)
 * Return TOPK_OK or TOPK_E_INVALID (unknown name / out of range). */
int topk_set_param(topk_ctx *ctx, const char *name, int64_t value);
int topk_get_param(const topk_ctx *ctx, const char *name, int64_t *value);

/* Bytes of device workspace a select call on n keys needs with the current
 * parameters.  The workspace needs no initialisation and may be reused by
 * later calls ordered on the same stream. */
size_t topk_workspace_bytes(const topk_ctx *ctx, uint64_t n, uint32_t flags);

/* Select the k smallest (largest with TOPK_LARGEST) of keys[0..n).
 *   keys      [n]  u32 or f32 keys
 *   n, k           1 <= k <= n < 2^32
 *   out_idx   [k]  positions of the selected keys, each exactly once, in an
 *                  unspecified order that may differ between calls (the
 *                  sweeps hand out output ranges in the order their
 *                  workgroups arrive); with TOPK_SORTED in the unique order
 *                  of Section 2: keys ascending (descending with
 *                  TOPK_LARGEST), ties by ascending position, NaN last
 *                  (first with TOPK_LARGEST), so out_idx[k-1] == kth_idx.
 *                  The order costs a radix sort of the k (order word,
 *                  position) pairs after the selection: about 16 k bytes of
 *                  traffic per pass, one pass per 8-bit digit that differs
 *                  among the pairs
 *   out_keys  [k]  NULL, or (with TOPK_WRITE_KEYS) keys[out_idx[i]], bits as in
 *                  the input (in out_idx's order, also with TOPK_SORTED)
 *   kth_key   [1]  the key of rank k (input bits, e.g. -0.0 and NaN payloads kept)
 *   kth_idx   [1]  its position; out_idx always contains it
 *   status    [1]  NULL or the device status word: TOPK_STATUS_OK, or
 *                  TOPK_STATUS_INTERNAL if a consistency check failed
 *   workspace      >= topk_workspace_bytes(ctx, n, flags) bytes, 256-byte aligned
 * Returns TOPK_OK, TOPK_E_INVALID, TOPK_E_WORKSPACE or TOPK_E_HIP. */
int topk_select_u32(topk_ctx *ctx, const uint32_t *keys, uint64_t n, uint64_t k,
                    uint32_t flags, uint32_t *out_idx, uint32_t *out_keys,
                    uint32_t *kth_key, uint32_t *kth_idx, uint32_t *status,
                    void *workspace, size_t ws_bytes, hipStream_t stream);
int topk_select_f32(topk_ctx *ctx, const float *keys, uint64_t n, uint64_t k,
                    uint32_t flags, uint32_t *out_idx, float *out_keys,
                    float *kth_key, uint32_t *kth_idx, uint32_t *status,
                    void *workspace, size_t ws_bytes, hipStream_t stream);

/* One recorded round of the last select call that used `workspace`
 * (§2 Algorithm: sample, pivots l = S[lo] and r = S[hi], counts of a and b).
 * The exact fallback round (after r_max attempts) has s = 0 and
 * lo = hi = TOPK_ROUND_EXACT: both pivots are the object of rank k_cur (a
 * sampled round always has hi >= 0; its lo < 0 means "no lower pivot"). */
#define TOPK_ROUND_EXACT (-2)
typedef struct topk_round_record {
    uint32_t n_cur, k_cur;   /* subproblem entering the round                    */
    uint32_t s;              /* sample size drawn                                 */
    uint32_t c_num;          /* spread factor used (c = c_num / 4)                */
    int64_t lo, hi;          /* pivot sample ranks (lo < 0: none; hi >= s: none) */
    uint32_t l_idx, r_idx;   /* pivot positions in the input (0 when absent)      */
    uint32_t has_l, has_r;
    uint32_t na, nb;         /* |a| = #{e < l}, |b| = #{l <= e <= r}               */
    uint32_t ok;             /* 1: recursed into b; 0: round repeated             */
    uint32_t tag;            /* attempt number = random stream of the round       */
} topk_round_record;

/* Copy the round records of the last select call out of `workspace` (device)
 * into `out` (host, room for `max` records); *count = rounds recorded.
 * Synchronises `stream`.  With TOPK_TRACE, *_trace_sample copies the sampled
 * objects (their input positions, in no particular order) of attempt `tag`
 * into out_pos (host, room for `cap`); *count = sample size. */
int topk_trace_rounds(const topk_ctx *ctx, const void *workspace, uint64_t n,
                      topk_round_record *out, uint32_t max, uint32_t *count,
                      hipStream_t stream);
int topk_trace_sample(const topk_ctx *ctx, const void *workspace, uint64_t n,
                      uint32_t tag, uint32_t *out_pos, uint32_t cap, uint32_t *count,
                      hipStream_t stream);

/* Kernel durations recorded (with parameter "timing" > 0) by the calls since
 * the last read-out, in enqueue order: ms[i] (milliseconds between HIP events
 * recorded on the call's stream just before and after the kernel) and
 * kind[i] (0 first pivot kernel, 1 pivot kernel, 2 first-round sweep,
 * 3 later sweep, 4 tail kernel).  Waits for the events; clears the record.
 * *count = kernels recorded (only min(count, max) are written). */
int topk_kernel_times(topk_ctx *ctx, float *ms, int32_t *kind, uint32_t max, uint32_t *count);

/* topk_tune_f32: the autotuner of the single-instance selection.  Same
 * arguments as topk_select_f32 without out_keys and status (flags:
 * TOPK_LARGEST only; the outputs are overwritten with valid results).  The
 * call is timed (mean of `reps` calls, HIP events on `stream`) under every
 * pair "s_target" in {2048, 4096, 8192} x "c_num" in {8, 12, 16, 24}, and
 * the fastest pair stays in ctx.  The workspace size does not depend on
 * either parameter.  Blocks the host until the stream is idle.  Returns
 * TOPK_OK, the errors of topk_select_f32, or TOPK_E_INVALID for reps outside
 * 1..100. */
int topk_tune_f32(topk_ctx *ctx, const float *keys, uint64_t n, uint64_t k, uint32_t flags,
                  uint32_t *out_idx, float *kth_key, uint32_t *kth_idx, void *workspace,
                  size_t ws_bytes, uint32_t reps, hipStream_t stream);

/* topk_stream_read: a measurement helper, not part of the selection.  Reads
 * keys[0 .. n) once with the column pattern of the first sweep (wave-tiles of
 * 64 columns x 64 lanes, 256-byte non-temporal loads; two 512-thread
 * workgroups per CU) and adds the sum of the key bits (mod 2^32) to *sink,
 * one atomic per workgroup, so that the plain stream-read bandwidth of the
 * device can be timed beside a selection.
 * keys 256-byte aligned, n a positive multiple of 4096; asynchronous on
 * `stream`.  Returns TOPK_OK, TOPK_E_INVALID or TOPK_E_HIP. */
int topk_stream_read(topk_ctx *ctx, const uint32_t *keys, uint64_t n, uint32_t *sink,
                     hipStream_t stream);

/* ---- Batched selection: many rows of uneven length, each with its own k ----
 *
 * topk_select_batched_f32: for every row r of a CSR batch, the k[r] smallest
 * (largest with TOPK_LARGEST) keys of keys[row_off[r] .. row_off[r+1]) under
 * the unique order by (key, column) of Section 2 (the same rule as
 * topk_select_f32, with column = position inside the row).
 *   keys     [row_off[rows]]  f32 keys of all rows, row after row
 *   row_off  [rows + 1]       u64 row boundaries (non-decreasing)
 *   k        [rows]           u32, 1 <= k[r] <= row length
 *   out_off  [rows + 1]       u64 exclusive prefix sums of k (caller-computed)
 *   out_idx  [out_off[rows]]  row r's selected columns at out_off[r] .. + k[r],
 *                             in an order fixed by the inputs, seed and
 *                             parameters (a short row, or one finished by the
 *                             exact fallback: column order)
 *   kth_key  [rows]           key of rank k[r] (bits as stored)
 *   kth_idx  [rows]           its column
 *   status   [1]              0, or TOPK_STATUS_BAD_ROW if some row had
 *                             k = 0, k > length or length >= 2^32 (skipped)
 *   workspace >= topk_batched_workspace_bytes(ctx, rows, flags), 256-aligned
 * One persistent launch of 256-thread workgroups over the rows, longest rows
 * first; each row by the sampling method with the workgroup as the machine
 * (batched.hip).  Context parameters tune it:
 *   "bt_s_target"  1024  expected sample size of a long row; 64..2048
 *   "bt_c_num"       12  pivot spread (as c_num above); 4..4096
 *   "bt_wg_per_cu"    4  resident workgroups per CU of the persistent grid; 1..8
 *   "bt_attempts"     4  sampling attempts before the exact fallback; 1..16
 *   "bt_tile"        16  keys per thread per step of the fast sweep: 8 or 16
 *                        (a tile of 2048 or 4096 keys)
 *   "bt_s_target@C", "bt_c_num@C", "bt_tile@C"  the same for the rows of length class C
 *                        only (lengths [2^(C-1), 2^C), 0 <= C < 34); -1
 *                        (default) falls back to the value above
 *   "bt_fast"         1  1: a row whose expected candidates (keys up to the
 *                        upper pivot) fit 0.7 of the workgroup's 4096 LDS
 *                        slots is swept once into per-wave LDS regions; 0:
 *                        always the general sweep (lower part straight to
 *                        out_idx, band to LDS)
 * flags: TOPK_LARGEST, TOPK_GRAPH
 * (capture the four launches into a hipGraph on first use for this exact
 * argument set and replay it afterwards; the ctx keeps up to 32 graphs and,
 * to make room for another, drains the device and drops one).  All
 * pointers are device pointers; asynchronous on `stream`.  Returns TOPK_OK,
 * TOPK_E_INVALID (null or misaligned pointer, rows = 0, unknown flag),
 * TOPK_E_WORKSPACE or TOPK_E_HIP. */
size_t topk_batched_workspace_bytes(const topk_ctx *ctx, uint32_t rows, uint32_t flags);
int topk_select_batched_f32(topk_ctx *ctx, const float *keys, const uint64_t *row_off,
                            uint32_t rows, const uint32_t *k, const uint64_t *out_off,
                            uint32_t flags, uint32_t *out_idx, float *kth_key,
                            uint32_t *kth_idx, uint32_t *status, void *workspace,
                            size_t ws_bytes, hipStream_t stream);

/* topk_select_batched_f32_noalloc: topk_select_batched_f32 for callers that
 * cannot allocate device memory or pass a workspace (code under HIP graph
 * capture, tight serving loops, harnesses that forbid allocation).  Same
 * arguments, results and kernels, without workspace and ws_bytes: the
 * workspace is a file-scope device array of the library (4 MiB + 70,144 bytes on
 * every device the library runs on, held until the process ends), enough for
 * rows <= 1,048,576.  No call allocates anything (no hipMalloc, no hipFree,
 * no allocating library routine); the library looks the array's device
 * address up once per device in topk_create.  Every call on a device shares
 * that array, and the launches clear what must start at zero: calls that
 * overlap on one device (different streams, or different host threads
 * without ordering) race and give undefined results.
 * flags: TOPK_LARGEST only (TOPK_GRAPH is rejected: the library would have
 * to create a stream and instantiate a graph; capture the call instead).
 * Returns TOPK_OK, TOPK_E_INVALID (as topk_select_batched_f32, or an unknown
 * flag), TOPK_E_WORKSPACE (rows > 1,048,576) or TOPK_E_HIP. */
int topk_select_batched_f32_noalloc(topk_ctx *ctx, const float *keys, const uint64_t *row_off,
                                    uint32_t rows, const uint32_t *k, const uint64_t *out_off,
                                    uint32_t flags, uint32_t *out_idx, float *kth_key,
                                    uint32_t *kth_idx, uint32_t *status, hipStream_t stream);

/* topk_tune_batched_f32: the autotuner of the batched form.  Same arguments
 * as topk_select_batched_f32 (TOPK_GRAPH ignored; the outputs are
 * overwritten with valid results).  For every length class of the batch whose
 * rows take the sampling path (longer than 8192 keys), the batch restricted to
 * that class is timed (mean of `reps` calls, HIP events on `stream`) under
 * each pair bt_s_target in {256, 512, 1024, 2048} x bt_c_num in
 * {8, 12, 16, 24}; the fastest pair becomes the class's "bt_s_target@C" /
 * "bt_c_num@C", and under it the faster of "bt_tile@C" in {8, 16}.  Then
 * "bt_attempts" in {1, 2, 4, 8} and "bt_wg_per_cu" in {2, 3, 4} are timed
 * over the whole batch and the fastest of each kept.  Blocks the host until the stream is idle.
 * Returns TOPK_OK, the errors of topk_select_batched_f32, or TOPK_E_INVALID
 * for reps outside 1..100. */
int topk_tune_batched_f32(topk_ctx *ctx, const float *keys, const uint64_t *row_off,
                          uint32_t rows, const uint32_t *k, const uint64_t *out_off,
                          uint32_t flags, uint32_t *out_idx, float *kth_key,
                          uint32_t *kth_idx, uint32_t *status, void *workspace,
                          size_t ws_bytes, uint32_t reps, hipStream_t stream);

/* Tuning files (host paths): a flat JSON object of "name": integer pairs,
 * the parameter names of topk_set_param ("seed" and "timing" excluded).
 * topk_save_tuning writes every tuning parameter and every length-class
 * override of ctx.  topk_load_tuning applies a file all or nothing (an unknown
 * name, a value out of range or a syntax error leaves ctx unchanged and
 * returns TOPK_E_INVALID); path NULL restores the built-in defaults.  Both
 * return TOPK_OK or TOPK_E_INVALID (also for a file that cannot be opened). */
int topk_save_tuning(const topk_ctx *ctx, const char *path);
int topk_load_tuning(topk_ctx *ctx, const char *path);

/* ---- Row-wise top-k (a differentiable layer's forward and backward) ----
 *
 * topk_rows_fwd_f32: for every row b of scores[B][N] (row-major, f32), the k
 * first elements of the row in selection order (the unique order by
 * (key, position) of Section 2, as for topk_select_f32; with TOPK_LARGEST
 * the largest keys first, NaN before everything), written in that order:
 *   values  [B][k]  key bits copied from scores (-0.0 and NaN payloads kept)
 *   indices [B][k]  column of each value (int64, the dtype torch.topk uses)
 * so values are descending with ties by ascending column (TOPK_LARGEST), or
 * ascending with ties by ascending column.  One workgroup per row: the
 * candidates at or before the k-th of the threads' local minima are ranked
 * exactly (see rows.hip); no workspace.  All pointers are device pointers;
 * the call is asynchronous on `stream`; ctx may be NULL.  Limits: 1 <= k <=
 * min(N, 1024), N <= 32768 (else TOPK_E_UNSUPPORTED).  flags: 0 or
 * TOPK_LARGEST.  Returns TOPK_OK, TOPK_E_INVALID (null or misaligned pointer,
 * B, N or k out of range, unknown flag), TOPK_E_UNSUPPORTED or TOPK_E_HIP. */
int topk_rows_fwd_f32(topk_ctx *ctx, const float *scores, uint32_t B, uint32_t N,
                      uint32_t k, uint32_t flags, float *values, int64_t *indices,
                      hipStream_t stream);

/* topk_scatter_bwd_f32: gradient of the row-wise top-k values with respect
 * to the scores: grad_in[b][j] = grad_out[b][m] where indices[b][m] = j, and
 * 0 elsewhere.  Every element of grad_in[B][N] is written exactly once (no
 * separate clearing).  indices as returned by topk_rows_fwd_f32 (distinct
 * within a row); entries outside [0, N) are ignored.  Device pointers,
 * asynchronous on `stream`.  Returns TOPK_OK, TOPK_E_INVALID (null or
 * misaligned pointer, B, N or k out of range), TOPK_E_UNSUPPORTED (more than
 * 2^31 - 1 workgroups) or TOPK_E_HIP. */
int topk_scatter_bwd_f32(const float *grad_out, const int64_t *indices, uint32_t B,
                         uint32_t N, uint32_t k, float *grad_in, hipStream_t stream);

/* ---- Top-k most frequent objects (§7) and top-k sum aggregation (§8) ----
 *
 * Objects are integers in [0, U).  One device stands in for the paper's PEs,
 * so the distributed hash table of §7.1 is a count table over [0, U) in the
 * workspace.  Context parameter "fq_mode" (0..3, default 0) picks how it is
 * filled; results are the same:
 *   direct (U <= 2^15 counting, 2^14 summing): every workgroup counts its
 *        range with one LDS counter per object, the rows are added up;
 *   partitioned (U <= 2^25): the (sampled) elements are split into
 *        partitions by the low bits of the object, every partition is counted
 *        with one LDS counter per object (no device atomic per element,
 *        whatever the skew);
 *   hashed: per-workgroup LDS hash tables (local aggregation) whose misses
 *        go straight to the table.
 * 0: the first that applies; 1: hashed; 2: partitioned where it applies,
 * else hashed; 3: as 0.
 * "Most frequent" follows the unique order of §2 with the count as the
 * value: larger counts first, ties by ascending object.
 *
 * topk_frequent_u32: the k most frequent objects of keys[0..n).
 *   keys      [n]  objects, each < U (others are skipped and flagged in
 *                  status); 16-byte aligned; 1 <= n < 2^32
 *   U              universe size, 1 <= U <= 2^31
 *   k              1 <= k <= min(U, 4096)
 *   kstar     0: Algorithm PAC (§7.1): Bernoulli sample, count the sampled
 *                  objects, select the k most frequently sampled;
 *             else Algorithm EC (§7.2), k <= kstar <= min(U, 4096): select
 *                  the kstar most frequently sampled, count those exactly
 *                  over the whole input, return the k most frequent of them
 *   T              sampling rate rho = T / 2^32, 1 <= T <= 2^32 (2^32:
 *                  every element); element i is sampled iff word i % 4 of
 *                  Philox4x32-10 at counter (i / 4, 0, 0, 2), key = the
 *                  context seed, is below T (topk_sample_threshold makes T
 *                  from a sample size)
 *   out_ids   [k]  the objects, most frequent first (ties: ascending object)
 *   out_counts[k]  PAC: their sample counts (the estimate of a count is
 *                  count * 2^32 / T); EC: their exact counts
 *   sample_counts [U]  NULL, or receives every object's sample count
 *   n_sampled [1]  NULL, or receives the sample size
 *   status    [1]  TOPK_STATUS_OK or TOPK_STATUS_BAD_KEY
 *   workspace      >= topk_frequent_workspace_bytes(ctx, n, U), 256-byte aligned
 *                  (partitioned counting: about 6 n bytes more)
 * Asynchronous on `stream`.  Returns TOPK_OK, TOPK_E_INVALID,
 * TOPK_E_WORKSPACE or TOPK_E_HIP. */
size_t topk_frequent_workspace_bytes(const topk_ctx *ctx, uint64_t n, uint32_t U);
int topk_frequent_u32(topk_ctx *ctx, const uint32_t *keys, uint64_t n, uint32_t U, uint32_t k,
                      uint32_t kstar, uint64_t T, uint32_t *out_ids, uint32_t *out_counts,
                      uint32_t *sample_counts, uint64_t *n_sampled, uint32_t *status,
                      void *workspace, size_t ws_bytes, hipStream_t stream);

/* topk_sum_top_u32: the k keys with the largest sums of values (§8).
 *   keys, values [n]  pairs (key < U, value >= 0), each array 16-byte aligned;
 *                  1 <= n < 2^32; the sum of all values must be < 2^63
 *   s              desired sample size, 1 <= s < 2^31.  The input is first
 *                  aggregated by key (sums[x]); with v_avg = m / s (m the
 *                  sum of all values) key x then yields floor(sums[x] /
 *                  v_avg) samples plus one with probability sums[x] / v_avg
 *                  minus that (word 0 of Philox4x32-10 at counter (x, 0, 0,
 *                  3), key = the context seed, below floor(r 2^32 / m), r =
 *                  sums[x] s mod m)
 *   kstar     0: PAC: the k keys with the most samples; out_vals = their
 *                  sample counts (estimate: count * m / s);
 *             else, k <= kstar <= min(U, 4096): the kstar keys with the most
 *                  samples, then the k largest of them by exact sum
 *                  (out_vals = exact sums)
 *   out_ids [k], out_vals [k]  keys (largest first, ties: ascending key), values
 *   sums [U], samples [U]      NULL, or receive the sums by key / the samples
 *   status    [1]  TOPK_STATUS_OK, TOPK_STATUS_BAD_KEY, TOPK_STATUS_SUM_RANGE
 *   workspace      >= topk_sum_workspace_bytes(ctx, n, U), 256-byte aligned
 *                  (partitioned counting: about 6 n bytes more)
 * Asynchronous on `stream`.  Returns TOPK_OK, TOPK_E_INVALID,
 * TOPK_E_WORKSPACE or TOPK_E_HIP. */
size_t topk_sum_workspace_bytes(const topk_ctx *ctx, uint64_t n, uint32_t U);
int topk_sum_top_u32(topk_ctx *ctx, const uint32_t *keys, const uint32_t *values, uint64_t n,
                     uint32_t U, uint32_t k, uint32_t kstar, uint64_t s, uint32_t *out_ids,
                     uint64_t *out_vals, uint64_t *sums, uint32_t *samples, uint32_t *status,
                     void *workspace, size_t ws_bytes, hipStream_t stream);

/* ---- Selection over sorted sequences (§4.2 / Appendix A, §4.3) ----
 *
 * The p sequences are the rows of a CSR batch: keys[row_off[r] ..
 * row_off[r + 1]) is row r, sorted ascending in the selection order (u32
 * unsigned; f32 as for topk_select_f32; TOPK_LARGEST: sorted descending, and
 * the largest are selected).  An object is identified by its position in
 * keys[], so ties go by ascending position, and the selected objects form a
 * prefix of every row: split[r] is that prefix's length.  Rows need not be
 * of equal length; some may be empty.  Limits: 1 <= p <= 8192, row_off[p] <
 * 2^32 (positions are 32-bit; checked on the device, which then writes
 * TOPK_STATUS_BAD_ARG and nothing else), keys 4-byte and row_off 8-byte
 * aligned.  One workgroup runs every round; the call is bound by the latency
 * of its binary searches, not by bandwidth.  No workspace.
 *
 * topk_msselect_*: Algorithm "musel" (quickselect over sorted sequences):
 * pivots uniform among the active objects (Philox4x32-10 at counter (round,
 * i, 0, 6), key = the context seed), located in every row by binary search;
 * d pivots per round (8 when p <= 1024, else 1; §4.3 "Multiple Concurrent
 * Trials"), recursion between the best pivot below rank k and the best above
 * (a pivot of rank exactly k ends it).  Writes split[p], *kth_pos (position of
 * the object of rank k), *kth_key (its bits), *rounds (NULL or the rounds
 * run), *status.  k in [1, n] (n = row_off[p] - row_off[0]).
 *
 * topk_amsselect_*: Algorithm "approxMusel": the k smallest objects for some
 * k in [kmin, kmax] (1 <= kmin <= kmax; kmax above n counts as n).  Each
 * round uses the min-based estimator (rate 1 - ((kmin-1)/kmax)^(1/(kmax-
 * kmin+1))) when kmin < n_cur - kmax, else the max-based one; every row draws
 * a geometric deviate per trial (Philox4x32-10 at counter (row, round, trial
 * / 4, 7)), the trial's pivot is the minimum (maximum) of the rows' sampled
 * objects, and the first trial whose count lies in [kmin, kmax] ends the
 * call; otherwise the recursion continues between the best trials below and
 * above.  After 64 rounds the call finishes exactly at rank kmin.  Writes
 * split[p], *k_out (= the sum of split), *rounds, *status.
 *
 * All asynchronous on `stream`.  Return TOPK_OK, TOPK_E_INVALID or TOPK_E_HIP. */
int topk_msselect_u32(topk_ctx *ctx, const uint32_t *keys, const uint64_t *row_off, uint32_t p,
                      uint64_t k, uint32_t flags, uint32_t *split, uint32_t *kth_pos,
                      uint32_t *kth_key, uint32_t *rounds, uint32_t *status, hipStream_t stream);
int topk_msselect_f32(topk_ctx *ctx, const float *keys, const uint64_t *row_off, uint32_t p,
                      uint64_t k, uint32_t flags, uint32_t *split, uint32_t *kth_pos,
                      float *kth_key, uint32_t *rounds, uint32_t *status, hipStream_t stream);
int topk_amsselect_u32(topk_ctx *ctx, const uint32_t *keys, const uint64_t *row_off, uint32_t p,
                       uint64_t kmin, uint64_t kmax, uint32_t flags, uint32_t *split,
                       uint64_t *k_out, uint32_t *rounds, uint32_t *status, hipStream_t stream);
int topk_amsselect_f32(topk_ctx *ctx, const float *keys, const uint64_t *row_off, uint32_t p,
                       uint64_t kmin, uint64_t kmax, uint32_t flags, uint32_t *split,
                       uint64_t *k_out, uint32_t *rounds, uint32_t *status, hipStream_t stream);

/* Sample sizes (host): the expected sample size for an (eps, delta)
 * approximation of §7 and §8 (0 < eps, 0 < delta < 1):
 *   TOPK_SAMPLE_PAC  4/eps^2 max(3/k ln(4n/delta), 2 ln(2k/delta))  (§7.1, equation
 *                    "sampleSize")
 *   TOPK_SAMPLE_EC   2/(eps^2 kstar) ln(n/delta)                    (§7.2, Lemma "topkec")
 *   TOPK_SAMPLE_SUM  (1/eps) sqrt(2 ln(2n/delta))                   (§8, proof of Theorem
 *                    "sumpac", one PE)
 * Returns -1 for invalid arguments.  topk_sample_threshold turns a sample
 * size into T = min(2^32, ceil(size 2^32 / n)) (at least 1). */
#define TOPK_SAMPLE_PAC 0
#define TOPK_SAMPLE_EC 1
#define TOPK_SAMPLE_SUM 2
double topk_sample_size(int method, uint64_t n, uint32_t k, uint32_t kstar, double eps,
                        double delta);
uint64_t topk_sample_threshold(uint64_t n, double sample_size);

const char *topk_strerror(int code);

#ifdef __cplusplus
}
#endif
#endif /* TOPK_H */
