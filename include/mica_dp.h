/*
 * mica_dp.h -- C ABI of the MI355X (gfx950) library for the dynamic-programming
 * phase of short-read alignment.
 *
 * What it computes (MICA paper, Methods, "Highly parallel dynamic
 * programming"): reads that few-mismatch search could not place are aligned
 * by DP allowing insertions and deletions (architecture section) against a
 * candidate region of the reference, with the affine gap model of three
 * tables M, I and D holding the best score of an alignment ending in a
 * Match, an Insert or a Delete.  Cell (i,j) of the table depends on
 * (i-1,j-1), (i-1,j) and (i,j-1).  DP serves reads that need gaps or clipped
 * ends, hence two modes: semi-global (the whole read against any substring
 * of the window) and local (both ends clipped, Smith-Waterman).
 *
 * Readings of what the paper leaves open (scores, boundaries, ties, CIGAR):
 *   - scoring: s(x,y) = match if x == y else mismatch; a gap of length L
 *     scores -(gap_open + L * gap_extend).
 *   - recurrences, 1 <= i <= m (read), 1 <= j <= n (window):
 *       D(i,j) = max(D(i,j-1) - e, H(i,j-1) - o - e)      (deletion)
 *       I(i,j) = max(I(i-1,j) - e, H(i-1,j) - o - e)      (insertion)
 *       H(i,j) = max(H(i-1,j-1) + s(q_i, r_j), D, I)  [and 0 when local]
 *   - semi-global boundary: H(0,j) = 0; H(i,0) = -(o + i*e); local: 0.
 *   - result cell: semi-global, the largest H(m,j) over 0 <= j <= n, ties to
 *     the smallest j; local, the largest H over all cells and (0,0), ties to
 *     the smallest j, then the smallest i.
 *   - traceback priorities: stop at H = 0 (local) > diagonal > D > I, and in
 *     a gap, opening it here beats extending it.
 *   - coordinates are 0-based, half-open and window-relative; CIGAR words are
 *     (length << 4) | op with M = 0, I = 1, D = 2 (BAM codes; no clipping ops:
 *     clipping is given by the start and end coordinates).
 *
 * Sequences are 2-bit packed: base codes A=0 C=1 G=2 T=3, base k of a buffer
 * at bits 2*(k % 16) of 32-bit word k / 16.  All positions and lengths are in
 * bases.
 *
 * Errors: every call returns a mica_status_t.  Batch-level problems (null
 * pointers, bad scoring or flags, sizes over the limits) return an error and
 * enqueue nothing.  Problems of a single pair are reported in that pair's
 * status word and the rest of the batch runs.  HIP failures return
 * MICA_ERR_HIP; mica_last_error() gives the text.  No C++ exception crosses
 * this interface.
 */
#ifndef MICA_DP_H
#define MICA_DP_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
  MICA_OK = 0,
  MICA_ERR_INVALID_ARG = -1,
  MICA_ERR_LIMIT = -2,
  MICA_ERR_OUT_OF_MEMORY = -3,
  MICA_ERR_HIP = -4,
  MICA_ERR_BUSY = -5
} mica_status_t;

/* Scoring: match > 0 and mismatch <= 0 are scores; gap_open >= 0 and
 * gap_extend >= 1 are penalties.  Limits: 1 <= match <= 4096,
 * -4096 <= mismatch <= 0, 0 <= gap_open <= 4096, 1 <= gap_extend <= 4096. */
typedef struct {
  int32_t match, mismatch, gap_open, gap_extend;
} mica_scoring_t;

/* Modes.  MICA_MODE_EXTEND is the read-extension use of DP with clipping:
 * the alignment is anchored at (0,0) with a start score h0 (the score of the
 * seed it extends; a leading gap at the anchor is an ordinary gap run), the
 * best early end is taken as in local mode with (0,0) worth h0, the best
 * end-to-end end as in semi-global mode on row m, and the read is aligned to
 * its end when that scores at least the early end minus the clipping
 * penalty (else it is clipped).  Starts are always (0,0). */
enum { MICA_MODE_SEMIGLOBAL = 0, MICA_MODE_LOCAL = 1, MICA_MODE_EXTEND = 2 };

/* flags of mica_dp_align_batch */
enum {
  MICA_OUT_START = 1u << 0,   /* write read_start and ref_start (runs the traceback) */
  MICA_OUT_CIGAR = 1u << 1,   /* write cigar and n_cigar (implies MICA_OUT_START) */
  MICA_FORCE_INT32 = 1u << 8, /* compute every pair with 32-bit scores */
  MICA_PLAIN_LAUNCH = 1u << 9, /* one launch per length bucket instead of the persistent one */
  MICA_NO_GRAPH = 1u << 10     /* enqueue the kernels one by one instead of as one HIP graph */
};

/* per-pair status bits */
enum {
  MICA_ST_SATURATED = 1u << 0,   /* 16-bit scores saturated; the 32-bit re-run result is final */
  MICA_ST_CIGAR_TRUNC = 1u << 1, /* n_cigar = -(runs needed); cigar holds the first cigar_cap runs */
  MICA_ST_LEN_LIMIT = 1u << 2,   /* m outside [min_read_len, max_read_len], n outside [0, max_win_len], mode not 0/1/2 (or outside mode_mask), or h0 out of range */
  MICA_ST_WIN_OOB = 1u << 3,     /* window not inside the reference: not computed */
  MICA_ST_READ_OOB = 1u << 4,    /* read not inside the read buffer: not computed */
  MICA_ST_INTERNAL = 1u << 5     /* a device consistency check failed; coordinates and CIGAR invalid */
};

#define MICA_MAX_READ_LEN 1024
#define MICA_MAX_WIN_LEN 8192

/* Library context: device workspace, plan table and launch cache for one
 * GPU.  Not thread-safe: use one context per host thread.  Calls that share
 * a context must be ordered on one stream (they share its workspace). */
typedef struct mica_ctx *mica_ctx_t;

/* Create a context on HIP device `hip_device`.  `workspace_bytes` caps the
 * device scratch the context may hold (0 = a default of 8 GiB); scratch is
 * allocated lazily and grown as batches need.  Writes the handle to *out. */
mica_status_t mica_ctx_create(int hip_device, size_t workspace_bytes, mica_ctx_t *out);

/* Free the context and its device memory (synchronises the device). */
mica_status_t mica_ctx_destroy(mica_ctx_t ctx);

/* One batch of independent (read, window) pairs.  Every pointer is a device
 * pointer owned by the caller; inputs must stay unchanged and outputs alive
 * until the work enqueued on the stream has completed. */
typedef struct {
  /* reference: 2-bit packed, ref_len bases */
  const uint32_t *ref2b;
  uint64_t ref_len;
  /* pair p aligns read p against ref[win_off[p], win_off[p] + win_len[p]) */
  const uint64_t *win_off;
  const int32_t *win_len;
  /* reads: 2-bit packed, reads_len bases; read p is reads[read_off[p], +read_len[p]) */
  const uint32_t *reads2b;
  uint64_t reads_len;
  const uint64_t *read_off;
  const int32_t *read_len;
  const uint8_t *mode; /* per pair MICA_MODE_*; NULL: every pair uses default_mode */
  int32_t default_mode;
  int64_t n_pairs;
  /* host-side upper bounds of read_len and win_len over the batch
   * (<= MICA_MAX_READ_LEN / MICA_MAX_WIN_LEN); they size the scratch and
   * choose the kernels.  A pair above them is not computed and gets
   * MICA_ST_LEN_LIMIT. */
  int32_t max_read_len, max_win_len;
  /* outputs (n_pairs entries each) */
  int32_t *score, *read_end, *ref_end; /* always written */
  int32_t *read_start, *ref_start;     /* required with MICA_OUT_START or MICA_OUT_CIGAR */
  uint32_t *cigar;                     /* n_pairs * cigar_cap words, required with MICA_OUT_CIGAR */
  int32_t cigar_cap;
  int32_t *n_cigar; /* required with MICA_OUT_CIGAR */
  uint32_t *status; /* always written */
  /* extension mode: start score per pair (NULL: ext_default_h0), 0..2^20,
   * and the clipping penalty, 0..2^20 */
  const int32_t *ext_h0;
  int32_t ext_default_h0;
  int32_t ext_clip;
  /* with a per-pair mode array: bit MICA_MODE_x set for every mode the
   * array may hold, 0 = any of the three.  Kernels of absent modes are not
   * launched; a pair whose mode is outside the mask gets MICA_ST_LEN_LIMIT.
   * Ignored without a mode array. */
  int32_t mode_mask;
  /* host-side lower bound of read_len over the batch (0 = none).  With the
   * upper bound it tells which read-length classes the batch can hold; a
   * batch of one class runs it as a plain launch.  A pair below it gets
   * MICA_ST_LEN_LIMIT. */
  int32_t min_read_len;
  /* host-side upper bound of the extension start scores (the ext_h0
   * entries, or ext_default_h0), 1..2^20; 0 = none given (2^20 assumed).
   * When every extension of the batch then provably stays inside 16-bit
   * scores, no saturation-checking kernels and no 32-bit re-run are
   * launched for it.  An extension pair above the bound gets
   * MICA_ST_LEN_LIMIT. */
  int32_t max_ext_h0;
} mica_batch_t;

/* Align every pair of `batch` (Methods, DP section; readings above).
 * Enqueues all work on `stream` (a hipStream_t; NULL = the null stream) and
 * returns without synchronising.  The result of every pair is exact: pairs
 * computed with 16-bit scores whose values reach the saturation guard band
 * are recomputed with 32-bit scores on the device (MICA_ST_SATURATED).
 * The kernels of one call (planning, fill, re-run) are one HIP graph launch:
 * the context builds a graph per distinct launch sequence on first use and
 * then only updates its grid sizes and parameter block (MICA_NO_GRAPH
 * launches the same kernels one by one). */
mica_status_t mica_dp_align_batch(mica_ctx_t ctx, const mica_batch_t *batch,
                                  const mica_scoring_t *scoring, uint32_t flags, void *stream);

/* ---- Allocation-free batch call -------------------------------------------
 * For callers that cannot allocate device memory: code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc.
 *
 * Same alignment, outputs and errors as mica_dp_align_batch (default plan,
 * kernels launched one by one, never a HIP graph), without a context: every
 * piece of device workspace (parameter block, bucket tables and counters,
 * per-pair work lists, traceback slots) lives in one fixed device array of
 * MICA_NOALLOC_SCRATCH_BYTES that each GPU the library runs on holds from
 * the first such call until the process ends.  The call itself allocates
 * and frees no device memory.  Runs on the calling thread's current HIP
 * device; the first call on a device looks up the array's address there.
 * Limits: at most MICA_NOALLOC_MAX_PAIRS pairs (MICA_ERR_LIMIT above), and
 * the traceback slots of one block of four waves must fit the array
 * (always true within MICA_MAX_READ_LEN / MICA_MAX_WIN_LEN); fewer waves
 * than the GPU could keep resident may run when windows are long.
 * The array is shared by every call on that GPU and keeps the last call's
 * contents: calls that overlap on one GPU (on any streams, from any
 * threads) race and give wrong results; order them on one stream or
 * synchronise between them.  Flags: MICA_OUT_START, MICA_OUT_CIGAR,
 * MICA_FORCE_INT32, MICA_PLAIN_LAUNCH (MICA_NO_GRAPH is accepted and has
 * no effect). */
#define MICA_NOALLOC_SCRATCH_BYTES ((size_t)256 << 20)
#define MICA_NOALLOC_MAX_PAIRS ((int64_t)1 << 22)
mica_status_t mica_dp_align_batch_noalloc(const mica_batch_t *batch, const mica_scoring_t *scoring,
                                          uint32_t flags, void *stream);

/* Pack n_bases base codes (one byte each, values 0..3) from device memory
 * `codes` into 2-bit words at device pointer `words` (ceil(n/16) words; the
 * unused high bits of the last word are zero).  Async on `stream`. */
mica_status_t mica_pack_2bit(const uint8_t *codes, int64_t n_bases, uint32_t *words, void *stream);

/* Kernel plan for reads of length in [m_lo, m_hi]: `lanes` lanes per pair
 * and `rows` read rows per lane, lanes * rows >= m_hi; (16, 1..16) or
 * (64, 4), (64, 8), (64, 16).  The default plan is (16, ceil(m/16)) up to 256
 * bases and (64, 16) above.  Lengths not covered keep their plan.  Plans
 * change only speed, never results.  Waits for all work on the device to
 * finish (batches already enqueued run with the plan they were enqueued
 * with), then copies the table to the device. */
mica_status_t mica_ctx_set_plan(mica_ctx_t ctx, int32_t m_lo, int32_t m_hi, int32_t lanes,
                                int32_t rows);

/* One read-length range of a tuned plan. */
typedef struct {
  int32_t m_lo, m_hi;  /* read lengths of the range */
  int32_t lanes, rows; /* plan chosen for it */
  int32_t n_pairs;     /* sample pairs in the range that were timed */
  int32_t n_candidates;
  int32_t n_rejected;  /* candidates whose outputs differed from the default plan's */
  int32_t pad_;
  double ms;           /* time of one call on the tuning batch with the range's choice */
  double default_ms;   /* the same before the range was tuned (its default plan) */
} mica_tune_entry_t;

/* Autotune the plan on a sample batch (same layout and flags as a batch of
 * mica_dp_align_batch; its output arrays are not written).  The tuning batch
 * is every sample pair of each 16-base read-length range (1-16, 17-32, ...)
 * with at least 256 pairs in the sample, up to 65,536 pairs per range.
 * Starting from the default plan, the ranges are tuned one at a time, the
 * earlier choices kept: each candidate plan of the range (16 lanes with the
 * fewest rows that cover it and one more row; 64 lanes with 4, 8 or 16 rows
 * where those cover it) is timed on the whole tuning batch (one warm-up,
 * then `reps` timed calls), because the plans of different ranges share
 * the launch (the persistent kernels balance the 16-lane plans against
 * each other, other plans run after them).  A candidate whose outputs
 * (every output array, every pair) differ from those of the default plan is
 * rejected; one that is more than 1% faster than the range's current choice
 * replaces it.  The context's plan table is left set to the choices.
 * Synchronises `stream`.  Writes up to out_cap entries to out (may be NULL;
 * ms and default_ms are whole-batch times after and before the range was
 * tuned) and their number to *n_out. */
mica_status_t mica_ctx_autotune(mica_ctx_t ctx, const mica_batch_t *sample, const mica_scoring_t *scoring,
                                uint32_t flags, void *stream, int32_t reps, mica_tune_entry_t *out,
                                int32_t out_cap, int32_t *n_out);

/* Save the context's plan table to a JSON file keyed by the device's
 * architecture name and compute-unit count; load it back into a context on
 * the same kind of device (another architecture or CU count is refused with
 * MICA_ERR_INVALID_ARG and leaves the plan unchanged). */
mica_status_t mica_ctx_save_plan(mica_ctx_t ctx, const char *path);
mica_status_t mica_ctx_load_plan(mica_ctx_t ctx, const char *path);

/* Counters of the last batch enqueued on ctx (synchronises `stream`). */
typedef struct {
  int64_t n_pairs;      /* pairs in the batch */
  int64_t n_items;      /* work items taken by the fill kernels */
  int64_t n_saturated;  /* pairs re-run with 32-bit scores */
  int64_t n_waves;      /* resident waves of the persistent launch */
  int64_t scratch_bytes;
  int64_t n_fallback;   /* pairs traced back from a full fill of direction bits (band too wide) */
  int64_t n_deferred;   /* pairs whose band (17-64 diagonals) was refilled by a later launch */
} mica_batch_stats_t;
mica_status_t mica_ctx_last_stats(mica_ctx_t ctx, void *stream, mica_batch_stats_t *out);

/* Kernel timing: with `enable` non-zero, every later mica_dp_align_batch
 * records a pair of HIP events on its stream around its fill launches (the
 * DP kernels proper, after planning).  mica_ctx_read_timing waits for the
 * recorded events, returns the summed fill time in milliseconds and the
 * number of timed batches since the previous read, and forgets them. */
mica_status_t mica_ctx_set_timing(mica_ctx_t ctx, int enable);
mica_status_t mica_ctx_read_timing(mica_ctx_t ctx, double *fill_ms, int64_t *n_batches);

/* ---- Serving ------------------------------------------------------------
 * A server keeps the reference resident on one GPU and aligns requests of
 * reads submitted from the host (the paper's host controller that feeds the
 * card large batches and keeps it busy, architecture section).  Each of the
 * in-flight slots has a host thread that takes every queued request that
 * fits (oldest first; up to 65,536 reads per batch) into its staging; each
 * slot has its own HIP stream, library context and staging, so host work,
 * copies and kernels of different slots overlap (continuous batching).  Requests whose staging
 * would not fit wait in the queue (admission by the slots' HBM budget).
 * Results are exact and identical to mica_dp_align_batch on the same pairs,
 * whatever else shares the batch.  All server calls are thread-safe. */
typedef struct mica_server *mica_server_t;

/* flag of mica_server_create: one request per batch (a FIFO baseline
 * without batching; use with max_inflight_slots = 1 for no overlap) */
enum { MICA_SERVE_FIFO = 1u << 16 };

/* Create a server on `hip_device`: uploads the 2-bit reference (host words,
 * ref_len bases) once; `hbm_budget_bytes` (0 = 24 GiB) bounds the device
 * memory of reference, slots' staging and their contexts' scratch (before
 * each batch a slot's context may grow into what the budget leaves after
 * the other slots' current workspaces, at least 64 MiB);
 * `max_inflight_slots` in 1..16; `flags`: mica_dp_align_batch flags
 * (MICA_OUT_CIGAR keeps 64 CIGAR runs per read) and MICA_SERVE_FIFO. */
mica_status_t mica_server_create(int hip_device, const uint32_t *host_ref2b, uint64_t ref_len,
                                 size_t hbm_budget_bytes, int max_inflight_slots,
                                 const mica_scoring_t *scoring, uint32_t flags, mica_server_t *out);

/* Seconds on the server's clock (a steady clock started at creation). */
mica_status_t mica_server_now(mica_server_t server, double *t);

/* Queue request `request_id` (unique among unfetched requests) of n reads:
 * read p is host_reads2b[read_off[p], +read_len[p]) (bases, 2-bit host
 * words), aligned against ref[win_off[p], +win_len[p]) in mode[p] (NULL: all
 * semi-global).  The arrays are copied before the call returns.
 * `arrival_time_s` on the server clock is the time latency is measured from
 * (< 0: now).  MICA_ERR_LIMIT for requests over 65,536 reads. */
mica_status_t mica_server_submit(mica_server_t server, uint64_t request_id, const uint32_t *host_reads2b,
                                 const uint64_t *read_off, const int32_t *read_len, const uint64_t *win_off,
                                 const int32_t *win_len, const uint8_t *mode, int64_t n,
                                 double arrival_time_s);

/* Replay a request schedule from a host thread inside the library (a load
 * generator that keeps up with high arrival rates): request r consists of
 * reads req_first[r] .. req_first[r] + req_count[r] - 1 of the given host
 * arrays (laid out as for mica_server_submit), gets id first_id + r and is
 * submitted at server time arrival_s[r] (the thread sleeps until then; the
 * latency of a request is measured from that time).  Returns at once; the
 * arrays must stay valid until mica_server_replay_wait returns.
 * MICA_ERR_BUSY while another replay runs. */
mica_status_t mica_server_replay(mica_server_t server, const uint32_t *host_reads2b, const uint64_t *read_off,
                                 const int32_t *read_len, const uint64_t *win_off, const int32_t *win_len,
                                 const uint8_t *mode, const int64_t *req_first, const int64_t *req_count,
                                 const double *arrival_s, int64_t n_requests, uint64_t first_id);

/* Wait until the replay has submitted every request; *lag_s (may be NULL)
 * gets how far the latest submission ran behind its scheduled time.  A
 * request the replay could not submit is reported here. */
mica_status_t mica_server_replay_wait(mica_server_t server, double *lag_s);

/* Ids of requests finished since the last poll (up to cap); *n_done of them. */
mica_status_t mica_server_poll(mica_server_t server, uint64_t *done_ids, int64_t cap, int64_t *n_done);

/* Copy a finished request's outputs (n entries each, as mica_dp_align_batch;
 * cigar: rows of cigar_cap words, of which the first min(|n_cigar|, 64,
 * cigar_cap) are written; any pointer may be NULL) and forget the request.
 * MICA_ERR_BUSY while it is not finished. */
mica_status_t mica_server_fetch(mica_server_t server, uint64_t request_id, int32_t *score,
                                int32_t *read_start, int32_t *read_end, int32_t *ref_start, int32_t *ref_end,
                                uint32_t *cigar, int32_t cigar_cap, int32_t *n_cigar, uint32_t *status);

/* Latency percentiles (finish - arrival, seconds) of the requests finished
 * since creation or the last reset, and their cells per second (GCUPS) over
 * the span from the first arrival to the last finish.  MICA_ERR_HIP if a
 * batch failed (its requests finish with MICA_ST_INTERNAL). */
mica_status_t mica_server_stats(mica_server_t server, double *p50_s, double *p99_s, double *gcups);
mica_status_t mica_server_reset_stats(mica_server_t server);

/* Give every slot's context a plan file (mica_ctx_save_plan; the kernel
 * plan per read-length range, e.g. tuned by mica_ctx_autotune on requests
 * like the expected ones; Methods, pipelining & load balancing).  Waits
 * until the queued and running batches have finished and holds submissions
 * meanwhile; later batches use the plan.  Results do not depend on the
 * plan.  MICA_ERR_INVALID_ARG for a file the contexts refuse (another
 * device kind, a malformed table). */
mica_status_t mica_server_load_plan(mica_server_t server, const char *path);

/* Finish the queued work, stop the worker and free everything. */
mica_status_t mica_server_destroy(mica_server_t server);

/* ---- Measurement -----------------------------------------------------------
 * Sustained integer VALU throughput of device `hip_device`, the roof the DP
 * fill kernels are bound by: every lane of 32 resident waves per compute
 * unit runs eight independent chains of add and max instructions, on packed
 * 16-bit pairs (*tops_i16x2, a packed instruction counting two operations)
 * and on 32-bit values (*tops_i32), in tera-operations per second.  Takes a
 * few milliseconds; synchronises the device. */
mica_status_t mica_measure_valu_peak(int hip_device, double *tops_i16x2, double *tops_i32);

/* Text of the last non-OK status returned on this host thread. */
const char *mica_last_error(void);

#ifdef __cplusplus
}
#endif

#endif /* MICA_DP_H */
