/*
 * mica_pipe.h -- C ABI of the host pipeline: FASTQ in, SAM out, both phases
 * of the aligner on one MI355X (gfx950).
 *
 * The paper's host controller feeds the card a million reads at a time,
 * keeps extra threads so that the card never waits, and emits SAM/BAM
 * (Methods: architecture & parallelism, pipelining & load balancing).  Here
 * one host thread parses FASTQ batches and packs them, one drives the GPU
 * and one or more format SAM records; the GPU work of a batch is:
 *   1. few-mismatch search of every read (include/mica_fm.h, k mismatches);
 *   2. for reads without a hit, one semi-global DP window per distinct seed
 *      placement of the search (window = placement -/+ band, clipped to the
 *      reference), all windows of the batch in one mica_dp_align_batch;
 *   3. per read, the best window (highest score, then the smallest
 *      reference start); its CIGAR words are compacted for the copy back.
 * Two slots (device buffers, stream, DP context) alternate between batches,
 * so the copies and kernels of one batch overlap the host work of the other.
 *
 * SAM records (one per read, in input order): reads found by the search are
 * written with CIGAR <m>M, NM = mismatches, AS = m*match + NM*(mismatch -
 * match), MAPQ 60 when the best mismatch count is unique, else 0; reads
 * placed by DP with the DP CIGAR, AS = the DP score, NM = mismatches plus gap
 * bases, MAPQ 60 when the best score is unique among the read's windows,
 * else 0, provided the score is at least min_score; every other read is
 * unmapped (flag 4): reads with bases other than ACGT, too short or too long
 * (search length limits), repetitive reads, reads with neither a hit nor a
 * DP window, reads whose best window scores below min_score or whose CIGAR
 * exceeds the staging capacity.
 */
#ifndef MICA_PIPE_H
#define MICA_PIPE_H

#include <stdint.h>

#include "mica_dp.h"

#ifdef __cplusplus
extern "C" {
#endif

typedef struct {
  int32_t k;             /* search mismatches, 0..2 */
  int32_t max_occ;       /* search repeat limit, 1..65536 */
  int32_t band;          /* DP window margin on each side of a seed placement, 0..3000 */
  int32_t min_score;     /* DP alignments scoring below it are unmapped */
  int32_t batch_reads;   /* reads per batch, 1..4,000,000 */
  int32_t format_threads; /* host threads formatting SAM records, 1..64 */
  mica_scoring_t scoring;
} mica_pipe_params_t;

typedef struct {
  int64_t reads, batches;
  int64_t mapped_search, mapped_dp, unmapped;
  int64_t non_acgt, repetitive;
  double seconds;       /* wall time of mica_pipe_run */
  double parse_seconds; /* reader thread busy time */
  double gpu_seconds;   /* GPU time of all batches (events) */
  double format_seconds;/* SAM formatting and writing busy time */
} mica_pipe_stats_t;

typedef struct mica_pipe *mica_pipe_t;

/* Build the pipeline on HIP device hip_device for a reference given as host
 * 2-bit words (ref_len bases, named ref_name in the SAM header): the FM index
 * (mica_fm_create), two DP contexts, two slots of device and pinned host
 * buffers sized for params->batch_reads reads of up to MICA_MAX_READ_LEN
 * bases.  The reference words are copied. */
mica_status_t mica_pipe_create(int hip_device, const uint32_t *host_ref2b, uint64_t ref_len, const char *ref_name,
                               const mica_pipe_params_t *params, mica_pipe_t *out);

/* Align every record of the FASTQ file and write SAM (header and one record
 * per read, in input order).  Either path may name a pipe: a regular input
 * file is mapped into memory for the run (it must not change meanwhile), a
 * regular output file is written at computed offsets, a pipe in order.
 * Returns MICA_ERR_INVALID_ARG for unreadable or malformed input (no output
 * is promised then); the pipeline stays usable.  One run at a time per
 * pipeline: the slots and contexts are its own. */
mica_status_t mica_pipe_run(mica_pipe_t pipe, const char *fastq_path, const char *sam_path,
                            mica_pipe_stats_t *stats);

mica_status_t mica_pipe_destroy(mica_pipe_t pipe);

#ifdef __cplusplus
}
#endif

#endif /* MICA_PIPE_H */
