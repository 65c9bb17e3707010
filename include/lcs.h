/*
 * lcs.h -- C ABI of liblcs_hip.so: exact longest-common-subsequence (LCS)
 * length and canonical LCS string on one AMD Instinct MI355X (gfx950).
 *
 * The operation is the dynamic program of Dash & Nayak, "Parallel Algorithm
 * for Longest Common Subsequence in a String" (arXiv:1306.4627):
 *
 *   section I.C (procedure LCS-length): with X = x_1..x_m indexing rows and
 *   Y = y_1..y_n indexing columns, c[i][0] = c[0][j] = 0 and
 *     c[i][j] = c[i-1][j-1] + 1                 if x_i == y_j   (DIAG)
 *             = c[i-1][j]   if c[i-1][j] >= c[i][j-1]           (UP)
 *             = c[i][j-1]   otherwise                           (LEFT)
 *   and the LCS length is c[m][n];
 *
 *   section I.D (procedure Print-LCS): start at (m, n); DIAG emits x_i and
 *   moves to (i-1, j-1), UP moves to (i-1, j), LEFT moves to (i, j-1); the
 *   emitted symbols, reversed, are the canonical LCS (ties go UP).
 *
 * The library computes exactly these values (bit-identical lengths and
 * strings); it never builds the tables.  Arguments are not symmetric for the
 * string: lcs_traceback(x, y) and lcs_traceback(y, x) may differ, the length
 * never does.  The returned string consists of bytes of X in forward order.
 *
 * Conventions for every entry point:
 *  - all pointers are HOST pointers unless the name says otherwise; the
 *    caller owns every buffer passed in and every buffer written to; nothing
 *    is returned that the caller must free except the opaque handles, which
 *    are released with their destroy call;
 *  - a sequence pointer may be NULL only when its length is 0;
 *  - on any negative status, no output buffer has been written;
 *  - m == 0 or n == 0 is valid (length 0, empty string);
 *  - calls on one context are not thread-safe; use one context per thread.
 */
#ifndef LCS_H_
#define LCS_H_

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
    LCS_PENDING = 1,          /* (request server) the request is queued or running */
    LCS_OK = 0,
    LCS_ERR_ARG = -1,         /* NULL pointer with non-zero length, bad flag or size */
    LCS_ERR_SYMBOL = -2,      /* a byte of X or Y is not in the alphabet */
    LCS_ERR_NOMEM = -3,       /* device memory budget or host memory exhausted */
    LCS_ERR_DEVICE = -4,      /* no usable gfx950 device, or a HIP runtime error */
    LCS_ERR_BUFFER = -5,      /* caller's output buffer is smaller than the worst case */
    LCS_ERR_TOO_LONG = -6,    /* a sequence is longer than LCS_MAX_LEN */
    LCS_ERR_UNSUPPORTED = -7  /* tuning request the library cannot honour */
} lcs_status;

/* Longest accepted sequence (|X| and |Y|), 2^31 - 1 symbols. */
#define LCS_MAX_LEN 2147483647ull

/* The alphabet of the input bytes (paper section I: DNA strands are strings
 * over {A, C, G, T}).  `size` is 1..256 and `symbols` lists `size` distinct
 * bytes; symbols == NULL with size == 256 means "every byte value".  Symbols
 * are compared as raw bytes (case-sensitive). */
typedef struct {
    uint16_t size;
    const uint8_t *symbols;
} lcs_alphabet;

/* One input pair: X (rows, length m) and Y (columns, length n). */
typedef struct {
    const uint8_t *x;
    uint64_t m;
    const uint8_t *y;
    uint64_t n;
} lcs_pair;

/* Opaque context: one device, one HIP stream, a device-memory budget. */
typedef struct lcs_ctx lcs_ctx;

/* Opaque resident batch: inputs uploaded once, run many times. */
typedef struct lcs_batch lcs_batch;

/* Batch flags. */
#define LCS_WANT_TRACEBACK 1u   /* also recover the canonical LCS of each pair */
#define LCS_USE_GRAPH      2u   /* replay the launch sequence as a HIP graph */
#define LCS_THRESHOLD      4u   /* threshold pass (lcs_batch_set_threshold); not
                                   with LCS_WANT_TRACEBACK */
#define LCS_FILL_TRACE     8u   /* record when every fill work item ran
                                   (lcs_batch_fill_trace) */

/* Length reported for a pair whose threshold answer came before its last
 * column (the fill of that pair stopped early). */
#define LCS_LENGTH_UNKNOWN UINT64_MAX

/* Tuning knobs; a zero field means "choose automatically".
 *  words_per_lane  : 64-bit words of the bit-vector column held per lane
 *                    (1, 2, 4 or 8);
 *  ckpt_interval   : columns between stored bit-vector checkpoints for the
 *                    traceback (64, 128 or 256; default 64);
 *  persistent_waves: cap on resident work-groups of the persistent kernels;
 *  plain           : 1 = no packing: one pair per work-group and one launch
 *                    per pair (the plain per-pair path, for comparison);
 *  strip_rows      : rows per traceback strip (rounded up to a multiple of
 *                    64*words_per_lane; default 4096).  The walk of a pair is
 *                    split into strips walked in parallel from estimated
 *                    entry columns and then reconciled; the result does not
 *                    depend on this value;
 *  tb_tiles        : checkpoint intervals per band the traceback
 *                    recomputes at once (1..8; default: about 256 columns
 *                    worth, fewer for wide bands);
 *  tb_bands        : bands the traceback recomputes at once (1..16,
 *                    tb_tiles * tb_bands <= 64; default: as many, up to 4,
 *                    as fit about 10 KiB of LDS per wave);
 *  link_items      : a pair too long for one wavefront continues in the
 *                    following work items, passing carries through memory;
 *                    it may start in the free lanes of the item before it
 *                    when the two need nearly the same number of column
 *                    steps.  Items linked this way form a run whose items all
 *                    wait on the one below; link_items caps a run's length
 *                    (default: 64 for traceback batches, whose fill the
 *                    6-8% fewer lane-steps make about 10% faster on the
 *                    4096-pair related batch; 1 -- a long pair always starts
 *                    a new item -- for lengths-only and threshold batches,
 *                    plain mode and traceback rounds).  Results do not
 *                    depend on it.
 *  tb_round_kib    : traceback history held at once, in KiB (0 = automatic).
 *                    The fast form stores the checkpoints and carry bits of
 *                    every work item during the fill, about m*n/64 bits per
 *                    pair.  With rounds the fill stores nothing but lengths
 *                    and the carry words handed between the items of a long
 *                    pair (16 bytes per 64 columns per 4096*words_per_lane
 *                    rows); the
 *                    items are then refilled round by round, top of each pair
 *                    first, each round keeping the history of at most
 *                    tb_round_kib KiB of items and walking the strips they
 *                    hold from where the previous round's walk left off.
 *                    Automatic: one pass when the whole history fits the
 *                    memory left, else rounds sized to what is left after the
 *                    batch's other buffers.  The history of one work item is
 *                    8*(words_per_lane+1) bytes per column (the smallest
 *                    round); results do not depend on it.
 *  halves          : lengths-only batches (no traceback, no threshold, not
 *                    plain): the length of a pair may be taken from two
 *                    fills of half its columns each, run side by side --
 *                    X against the first h = floor(n/2) symbols of Y, and X
 *                    reversed against the rest of Y reversed -- as the
 *                    largest sum, over the rows k, of the first half's
 *                    c[k][h] and the second half's LCS of the last m - k
 *                    symbols of X with the rest of Y (section I.C's table
 *                    cut at column h, the middle-column split Hirschberg's
 *                    method is built on).  A pair's column steps, the
 *                    latency of its fill, halve; its cells stay the same.
 *                    0 = automatic: split pairs of at least 4096 x 4096
 *                    symbols when the batch at one word per lane, split,
 *                    takes at most a quarter of the device's resident lanes
 *                    (a batch too small to fill the device waits on its
 *                    longest pair); 1 = never; 2 = every pair with n >= 2.
 *                    Ignored for other batches; results do not depend on it. */
typedef struct {
    int32_t words_per_lane;
    int32_t ckpt_interval;
    int32_t persistent_waves;
    int32_t plain;
    int32_t strip_rows;
    int32_t tb_tiles;
    int32_t tb_bands;
    int32_t link_items;
    int32_t tb_round_kib;
    int32_t halves;
} lcs_tuning;

/* What a batch was planned into (filled by lcs_batch_info). */
typedef struct {
    uint64_t pairs;          /* pairs in the batch */
    uint64_t cells;          /* sum of m*n over the pairs */
    uint64_t groups;         /* packed work items (all classes) */
    uint64_t lanes;          /* lanes of all work items, busy or idle */
    uint64_t lane_steps;     /* sum over work items of lanes * steps */
    uint64_t device_bytes;   /* device memory held by the batch */
    int32_t words_per_lane;  /* as chosen */
    int32_t ckpt_interval;   /* as chosen (0 without traceback) */
    int32_t classes;         /* kernel launches per run (fill) */
    int32_t flags;           /* LCS_WANT_TRACEBACK / LCS_USE_GRAPH as planned */
    int32_t tb_rounds;       /* traceback rounds (0: one pass, full history) */
    int32_t split_pairs;     /* pairs whose length comes from two half fills
                                (lcs_tuning.halves) */
    uint64_t history_bytes;  /* device bytes of traceback history (checkpoints
                                and carry bits, or the round buffer) */
} lcs_batch_stats;

/* Text for a status code; never NULL; static storage. */
const char *lcs_status_str(int status);

/* Library version string; static storage. */
const char *lcs_version(void);

/* Text of the last HIP runtime error or kernel failure seen by this thread
 * ("" if none); thread-local storage, valid until the next call. */
const char *lcs_last_error(void);

/* Create a context on HIP device `device`.  mem_budget_bytes caps the device
 * memory the context's batches may hold (0 = 90% of the device's free memory
 * at creation).  Returns LCS_ERR_DEVICE when the device is absent or is not a
 * gfx950 part.  *out is written only on success. */
lcs_status lcs_create(lcs_ctx **out, int device, size_t mem_budget_bytes);

/* Release a context and everything it holds (NULL is ignored).  Batches
 * created on it must have been destroyed first. */
void lcs_destroy(lcs_ctx *ctx);

/* Make subsequent work of `ctx` run on `hip_stream` (a hipStream_t of the
 * context's device, e.g. torch.cuda.current_stream().cuda_stream on ROCm);
 * NULL selects the context's own stream.  The caller keeps the stream alive. */
lcs_status lcs_set_stream(lcs_ctx *ctx, void *hip_stream);

/* The context's device as the runtime reports it: compute units and peak
 * shader clock in kHz (either pointer may be NULL).  The roofline of the
 * fill is compute_units * 64 lanes * clock * 64 cells / 6 instructions. */
lcs_status lcs_device_info(lcs_ctx *ctx, int32_t *compute_units, int32_t *peak_clock_khz);

/* Wait for all work queued on the context's stream. */
lcs_status lcs_synchronize(lcs_ctx *ctx);

/* LCS length of one pair (section I.C: c[m][n]).  Blocks until done. */
lcs_status lcs_length(lcs_ctx *ctx, const uint8_t *x, uint64_t m,
                      const uint8_t *y, uint64_t n, const lcs_alphabet *alphabet,
                      uint64_t *out_len);

/* Canonical LCS of one pair (sections I.C and I.D).  `out` receives
 * *out_len bytes of X in forward order; out_cap must be >= min(m, n)
 * (LCS_ERR_BUFFER otherwise).  Blocks until done. */
lcs_status lcs_traceback(lcs_ctx *ctx, const uint8_t *x, uint64_t m,
                         const uint8_t *y, uint64_t n, const lcs_alphabet *alphabet,
                         uint8_t *out, uint64_t out_cap, uint64_t *out_len);

/* LCS lengths of `count` pairs, one packed persistent launch per class.
 * out_lens[k] is the length of pairs[k].  Blocks until done. */
lcs_status lcs_length_batch(lcs_ctx *ctx, const lcs_pair *pairs, uint64_t count,
                            const lcs_alphabet *alphabet, uint64_t *out_lens);

/* Canonical LCS of `count` pairs.  The strings are written back to back into
 * out_arena: pair k occupies out_lens[k] bytes at out_offsets[k].  arena_cap
 * must be >= sum over pairs of min(m, n) (LCS_ERR_BUFFER otherwise).  Blocks
 * until done. */
lcs_status lcs_traceback_batch(lcs_ctx *ctx, const lcs_pair *pairs, uint64_t count,
                               const lcs_alphabet *alphabet, uint8_t *out_arena,
                               uint64_t arena_cap, uint64_t *out_offsets,
                               uint64_t *out_lens);

/* Allocation-free form of lcs_traceback_batch, for callers that cannot
 * allocate device memory (code inside HIP graph capture, tight serving loops,
 * harnesses that forbid hipMalloc).  Same arguments, results and errors as
 * lcs_traceback_batch; every byte of device memory the batch needs (inputs,
 * plan tables, checkpoints, bitmaps, queue counters, outputs before the copy
 * back) is carved from one fixed array of lcs_noalloc_scratch_bytes() bytes
 * that each device holds from library load until the process ends.  Calls no
 * hipMalloc/hipFree and creates no HIP objects; uses the context's stream and
 * blocks until done.  A batch whose full traceback history would not fit the
 * array runs its traceback in rounds (see lcs_tuning.tb_round_kib); one that
 * needs more than the array even so fails with LCS_ERR_NOMEM before any
 * launch (lcs_last_error() names both sizes).  Calls
 * on one device share its array: they are serialised inside the process (a
 * call holds the device's array until its results are copied back), and
 * every pass clears what must start at zero. */
lcs_status lcs_traceback_batch_noalloc(lcs_ctx *ctx, const lcs_pair *pairs, uint64_t count,
                                       const lcs_alphabet *alphabet, uint8_t *out_arena,
                                       uint64_t arena_cap, uint64_t *out_offsets,
                                       uint64_t *out_lens);

/* Size in bytes of the fixed scratch array of lcs_traceback_batch_noalloc. */
uint64_t lcs_noalloc_scratch_bytes(void);

/* Plan and upload a batch without running it.  The input bytes are copied to
 * device memory; the caller's host buffers may be released afterwards.
 * flags: LCS_WANT_TRACEBACK | LCS_USE_GRAPH | LCS_THRESHOLD | LCS_FILL_TRACE.
 * tuning may be NULL (automatic).
 * Fails with LCS_ERR_NOMEM when the batch would exceed the context budget. */
lcs_status lcs_batch_create(lcs_ctx *ctx, const lcs_pair *pairs, uint64_t count,
                            const lcs_alphabet *alphabet, uint32_t flags,
                            const lcs_tuning *tuning, lcs_batch **out);

/* Enqueue one full pass (symbol remap, match masks, fill, length and, if
 * planned, traceback) on the context's stream.  Asynchronous; inputs stay
 * resident, so repeated runs recompute from the same device data. */
lcs_status lcs_batch_run(lcs_batch *batch);

/* Wait for the batch's last run and copy its lengths (input order). */
lcs_status lcs_batch_lengths(lcs_batch *batch, uint64_t *out_lens);

/* Wait for the batch's last run and copy its strings, laid out as in
 * lcs_traceback_batch.  LCS_ERR_ARG if the batch was planned without
 * LCS_WANT_TRACEBACK. */
lcs_status lcs_batch_tracebacks(lcs_batch *batch, uint8_t *out_arena, uint64_t arena_cap,
                                uint64_t *out_offsets, uint64_t *out_lens);

/* Describe how the batch was planned. */
lcs_status lcs_batch_info(const lcs_batch *batch, lcs_batch_stats *out);

/* Run the batch once, wait for it and report HIP-event timings (inputs
 * already resident).  eager == 0 runs it as lcs_batch_run does (a graph
 * replay if planned with LCS_USE_GRAPH); eager != 0 enqueues the kernels
 * directly, which also times the fill kernels on their own.  *total_ms
 * receives the duration of the whole pass, *fill_ms that of the fill kernels
 * alone, or -1 for a graph replay; either pointer may be NULL. */
lcs_status lcs_batch_time(lcs_batch *batch, int eager, float *total_ms, float *fill_ms);

/* Shader clock during the batch's last fill launch, in MHz: the shader-cycle
 * counter over the 100 MHz counter, both read by the fill's first wave when
 * it starts and when it finds no more work (so: the clock while the fill
 * ran at full load).  LCS_ERR_ARG before the first run; LCS_ERR_DEVICE if
 * the counters did not advance. */
lcs_status lcs_batch_clock(lcs_batch *batch, double *mhz);

/* Schedule record of one fill work item (64 lanes' share of the column
 * steps, run by one wavefront from the persistent queue) in the last pass of a
 * batch created with LCS_FILL_TRACE.  Times are nanoseconds after the earliest
 * item of the pass was taken, from the GPU's 100 MHz counter (10 ns
 * resolution). */
typedef struct {
    uint64_t start_ns;       /* taken from the queue */
    uint64_t first_step_ns;  /* match masks built; first column step */
    uint64_t end_ns;         /* after the last column step */
    uint64_t wait_ns;        /* spent waiting for the carries of its feeder */
    uint32_t steps;          /* column steps of the item */
    int32_t feeder;          /* index of the item that hands it carries, -1 if none */
    uint32_t feeds;          /* 1 when it hands carries to the next item */
    uint32_t ran;            /* 0 when the pass never took it (a failed pass) */
    uint32_t hw_id;          /* HW_ID of the wavefront that ran it: wave slot
                                (bits 0-3), SIMD (4-5), CU (8-11), shader array
                                (12), shader engine (13-15) */
    uint32_t xcc_id;         /* XCC_ID: the accelerator die (bits 0-3) */
} lcs_fill_item;

/* Schedule records of the batch's last pass, one per fill work item in queue
 * order (all classes).  *count receives the number of items; with out NULL
 * only the count is returned.  LCS_ERR_ARG if the batch was created without
 * LCS_FILL_TRACE, before its first run, or if cap < *count.  The records cost
 * the fill a few stores per item; keep the flag off for timed runs. */
lcs_status lcs_batch_fill_trace(lcs_batch *batch, lcs_fill_item *out, uint64_t cap,
                                uint64_t *count);

/* Release a batch (NULL is ignored). */
void lcs_batch_destroy(lcs_batch *batch);

/* ---- derived outputs (section II) -----------------------------------------
 *
 * Section II asks whether a child sequence carries the characteristics of
 * its parent, and by what percentage.  Here X is the parent and Y the child,
 * and the similarity of a pair is the share of the parent its LCS keeps:
 * (100 * L) / m in double precision (the product is exact; one rounding in
 * the division), and 100 when m == 0.  The yes/no form asks whether the
 * similarity is at least a given percentage; it is settled as soon as the
 * partial columns prove it either way, so the fill of such a pair stops
 * early (lengths are then not known).  Each pair's answer depends on the
 * pair alone and is exact: it equals the comparison made on the full
 * length. */

/* Similarity percentages of `count` pairs (out_percent[k] for pairs[k]),
 * from their exact lengths.  Blocks until done. */
lcs_status lcs_similarity_batch(lcs_ctx *ctx, const lcs_pair *pairs, uint64_t count,
                                const lcs_alphabet *alphabet, double *out_percent);

/* Threshold answers of `count` pairs: out_pass[k] = 1 when the similarity of
 * pairs[k] is at least min_percent (0 <= min_percent <= 100, LCS_ERR_ARG
 * otherwise, NaN included), else 0.  out_len (may be NULL) receives each
 * pair's length when its fill ran to the last column, LCS_LENGTH_UNKNOWN when
 * the answer came earlier.  Blocks until done. */
lcs_status lcs_threshold_batch(lcs_ctx *ctx, const lcs_pair *pairs, uint64_t count,
                               const lcs_alphabet *alphabet, double min_percent,
                               uint8_t *out_pass, uint64_t *out_len);

/* Set the threshold of a batch created with LCS_THRESHOLD (required before
 * its first run; may be changed between runs).  Each pair's target length
 * -- the least L whose similarity reaches min_percent -- is computed on the
 * host in double precision and copied to the device on the batch's stream.
 * LCS_ERR_ARG for a batch without LCS_THRESHOLD or min_percent outside
 * [0, 100]. */
lcs_status lcs_batch_set_threshold(lcs_batch *batch, double min_percent);

/* Wait for the batch's last run and copy its threshold answers (out_pass,
 * input order, 1 = reaches the threshold) and lengths (out_len, may be NULL;
 * LCS_LENGTH_UNKNOWN for pairs answered before their last column).
 * LCS_ERR_ARG for a batch without LCS_THRESHOLD.  lcs_batch_lengths on such
 * a batch reports the same lengths. */
lcs_status lcs_batch_decisions(lcs_batch *batch, uint8_t *out_pass, uint64_t *out_len);

/* Timed search for the tuning of a batch (the batched form's autotuner).
 * Plans and runs the batch (flags as for lcs_batch_create) under candidate
 * tunings -- words_per_lane 1, 2, 4, 8 as the alphabet allows, then with
 * LCS_WANT_TRACEBACK the checkpoint interval 64 or 128 and the tiles per
 * traceback round -- and writes the fastest to *best and its pass time (ms,
 * graph replay when LCS_USE_GRAPH is set) to *best_ms (may be NULL).  Each
 * candidate uploads the inputs and runs three passes; results are not kept.
 * The answer is cached in the context under the batch's shape (flags,
 * alphabet size, and log2 of the pair count, of the longest X and Y and, in
 * quarters, of the total cells); a later call with a batch of the same shape
 * returns it without running anything.  Candidates that do not fit the
 * memory budget are skipped; LCS_ERR_NOMEM if none fits.  Argument and
 * symbol errors as for lcs_batch_create; LCS_THRESHOLD is not accepted
 * (tune the lengths-only shape and pass its tuning to lcs_batch_create). */
lcs_status lcs_autotune(lcs_ctx *ctx, const lcs_pair *pairs, uint64_t count,
                        const lcs_alphabet *alphabet, uint32_t flags, lcs_tuning *best,
                        float *best_ms);

/* ---- request server (continuous batching) --------------------------------
 *
 * A server accepts single LCS requests at any time and answers each one
 * exactly as lcs_length / lcs_traceback would.  A dispatcher thread of its
 * own gathers the requests waiting in arrival order -- the oldest one and
 * the later ones with the same alphabet and traceback choice -- into a batch
 * whenever one of its streams is free, and launches it while earlier
 * batches still run, so requests that arrive during other work are admitted
 * as streams and memory free up and their work overlaps on the device.
 * Device memory for the resident requests (sequences, match masks,
 * checkpoints, bitmaps) comes from one arena reserved from the context's
 * budget at creation; a batch that does not fit the free arena is retried
 * smaller or waits for running batches, and a request that cannot fit the
 * empty arena fails with LCS_ERR_NOMEM.  Inputs are copied at submission;
 * results stay with the server until lcs_result collects them.  While a
 * server runs, its context may still be used for other calls from the
 * caller's thread (other streams, other memory). */
typedef struct lcs_server lcs_server;

typedef struct {
    size_t mem_budget_bytes;   /* arena size; 0 = half of what the context budget has left */
    int32_t streams;           /* batches in flight at once, 1..16 (0 = 4) */
    int32_t max_batch_pairs;   /* requests per batch (0 = 4096) */
} lcs_server_config;

typedef struct {
    uint64_t submitted, completed, failed, cancelled;
    uint64_t queued;           /* waiting for admission now */
    uint64_t batches;          /* batches launched */
    uint64_t max_inflight;     /* most batches running at once */
    uint64_t cells;            /* sum of m*n over completed requests */
    uint64_t arena_bytes, arena_peak_bytes;
    uint64_t plan_ns;          /* dispatcher time planning, uploading and launching batches */
    uint64_t collect_ns;       /* dispatcher time copying finished batches' results */
    uint64_t device_ns;        /* sum over batches of launch-to-completion time */
    uint64_t tuned_batches;    /* batches launched with a tuning the context's
                                  autotuner cache held for their shape */
} lcs_server_stats;

/* Start a server on the context (cfg may be NULL for the defaults). */
lcs_status lcs_server_create(lcs_ctx *ctx, const lcs_server_config *cfg, lcs_server **out);

/* Stop accepting requests, drop the queued ones, let running batches
 * finish, release the arena and the streams (NULL is ignored). */
void lcs_server_destroy(lcs_server *server);

/* Queue one request (X, Y validated against the alphabet now; the bytes are
 * copied).  want_traceback != 0 also recovers the canonical LCS string.
 * *ticket names the request in the calls below. */
lcs_status lcs_submit(lcs_server *server, const uint8_t *x, uint64_t m, const uint8_t *y,
                      uint64_t n, const lcs_alphabet *alphabet, int want_traceback,
                      uint64_t *ticket);

/* LCS_PENDING while queued or running, LCS_OK when done, else the status the
 * request failed with; LCS_ERR_ARG for an unknown ticket. */
lcs_status lcs_poll(lcs_server *server, uint64_t ticket);

/* As lcs_poll, after waiting up to timeout_us microseconds (< 0: no limit)
 * for the request to finish. */
lcs_status lcs_wait(lcs_server *server, uint64_t ticket, int64_t timeout_us);

/* Collect a finished request: *len its LCS length, out (capacity out_cap)
 * its LCS string when a traceback was requested, *latency_ns (may be NULL)
 * the time from submission to completion.  Releases the ticket, also when
 * the request failed (its status is returned).  LCS_PENDING if not finished;
 * LCS_ERR_BUFFER (ticket kept) if out_cap is smaller than the string. */
lcs_status lcs_result(lcs_server *server, uint64_t ticket, uint64_t *len, uint8_t *out,
                      uint64_t out_cap, uint64_t *latency_ns);

/* Withdraw a request that is still queued (LCS_ERR_ARG otherwise). */
lcs_status lcs_cancel(lcs_server *server, uint64_t ticket);

/* Counters since creation. */
lcs_status lcs_server_stats_get(lcs_server *server, lcs_server_stats *out);

/* Host-only planning check (no device needed).  Packs `count` pairs of the
 * given lengths for `words_per_lane` and reports the same figures
 * lcs_batch_info would (device_bytes excluded).  Used to test the packer. */
lcs_status lcs_plan_describe(const uint64_t *m, const uint64_t *n, uint64_t count,
                             uint16_t alphabet_size, uint32_t flags,
                             const lcs_tuning *tuning, lcs_batch_stats *out);

/* Host-only: validate the packer's lane assignment for the given lengths --
 * every pair covered by exactly ceil(ceil(m/64)/words_per_lane) consecutive
 * lanes of one work item, no lane shared, every carry hand-over in bounds.
 * Returns LCS_OK when all checks hold, LCS_ERR_ARG otherwise. */
lcs_status lcs_plan_selfcheck(const uint64_t *m, const uint64_t *n, uint64_t count,
                              uint16_t alphabet_size, uint32_t flags,
                              const lcs_tuning *tuning);

#ifdef __cplusplus
}
#endif

#endif /* LCS_H_ */
