/*
 * mica_fm.h -- C ABI of the few-mismatch search phase on one MI355X (gfx950).
 *
 * The aligner's first phase places each read with few mismatches through a
 * BWT (FM) index of the reference held in device memory, and hands the reads
 * it cannot place to the DP phase (Methods: architecture & parallelism; the
 * BWT queries are the other hot loop named under extra parallelism).
 *
 * What is computed, per read of m bases against a reference of L bases
 * (forward strand, one sequence) with at most k <= 2 mismatches:
 *   hits = { p : 0 <= p <= L - m, Hamming(read, ref[p, p + m)) <= k }
 *   best_mm = min mismatches over hits (-1 without hits), n_best = hits with
 *   best_mm mismatches, n_hits = |hits|, pos = the smallest hit position with
 *   best_mm mismatches (-1 without hits).
 * How: the read is cut into k + 1 parts, part j = [floor(j m/(k+1)),
 * floor((j+1) m/(k+1))); every hit has an exact part (pigeonhole).  Each part
 * is searched exactly by backward search in the FM index, its occurrences are
 * read from the suffix array and each candidate placement is verified on the
 * 2-bit reference; a hit is counted by its lowest-index exact part only.
 * A read with a part that occurs more than max_occ times is not searched
 * (MICA_ST_REPETITIVE), standing for the paper's threads leaving repetitive
 * reads to the host.
 *
 * All functions return MICA_OK (0) or a negative mica_status_t;
 * mica_last_error() describes the last failure of the calling thread.
 */
#ifndef MICA_FM_H
#define MICA_FM_H

#include <stddef.h>
#include <stdint.h>

#include "mica_dp.h"

#ifdef __cplusplus
extern "C" {
#endif

/* Per-read status bit of the search (in addition to MICA_ST_LEN_LIMIT for
 * m < k + 1 or m > MICA_MAX_READ_LEN and MICA_ST_READ_OOB). */
#define MICA_ST_REPETITIVE (1u << 6)

#define MICA_FM_MAX_REF_LEN 4294967290ull /* suffix array entries are 32-bit */
#define MICA_FM_MAX_OCC 65536

/* Suffix array of codes[0, n) followed by a sentinel smaller than every code
 * (codes 0..3): sa[0, n] receives the n + 1 suffix starts in lexicographic
 * order, so sa[0] = n.  Host memory, caller-owned; SA-IS (induced sorting),
 * linear time, single thread.  Fails for n > MICA_FM_MAX_REF_LEN or a code
 * above 3. */
mica_status_t mica_fm_suffix_array(const uint8_t *codes, uint64_t n, uint32_t *sa);

typedef struct mica_fm *mica_fm_t;

/* Build the FM index of a reference given as host 2-bit words (ref_len
 * bases, base k of a word at bits 2(k mod 16)) and upload it to HIP device
 * hip_device: occurrence blocks (64 B per 192 BWT symbols: four 32-bit counts
 * and twelve words of 2-bit symbols), the full 32-bit suffix array and a
 * padded copy of the reference.  The build runs on the calling host thread;
 * the device memory stays allocated until mica_fm_destroy. */
mica_status_t mica_fm_create(int hip_device, const uint32_t *host_ref2b, uint64_t ref_len, mica_fm_t *out);

/* Free the index (synchronises the device). */
mica_status_t mica_fm_destroy(mica_fm_t fm);

/* Device bytes held by the index and host seconds its build took. */
mica_status_t mica_fm_info(mica_fm_t fm, uint64_t *device_bytes, double *build_seconds);

/* One batch of reads.  Every pointer is a device pointer owned by the
 * caller; inputs must stay unchanged and outputs alive until the work
 * enqueued on the stream has completed. */
typedef struct {
  const uint32_t *reads2b; /* 2-bit packed reads, reads_len bases */
  uint64_t reads_len;
  const uint64_t *read_off; /* read r is reads[read_off[r], + read_len[r]) */
  const int32_t *read_len;
  int64_t n_reads;
  int32_t k;       /* 0..2 mismatches */
  int32_t max_occ; /* 1..MICA_FM_MAX_OCC occurrences per part */
  /* outputs, n_reads entries each, always written */
  int32_t *best_mm, *n_best, *n_hits;
  int64_t *pos;
  uint32_t *status;
  /* optional (NULL: not written): 3 entries per read, entry j the smallest
   * placement (occurrence start minus the part's offset in the read) among
   * the exact occurrences of part j, for j <= k when the part occurs at most
   * max_occ times; MICA_FM_NO_CAND otherwise.  Placements may lie partly
   * outside the reference.  These are the seeds of the DP windows of reads
   * without a hit. */
  int64_t *cand;
} mica_fm_batch_t;

#define MICA_FM_NO_CAND INT64_MIN

/* Search every read of the batch (one kernel launch on the caller's
 * hipStream_t; asynchronous, allocates nothing).  The index is read only:
 * calls from several host threads or on several streams may overlap. */
mica_status_t mica_fm_search(mica_fm_t fm, const mica_fm_batch_t *batch, void *stream);

#ifdef __cplusplus
}
#endif

#endif /* MICA_FM_H */
