/*
 * CPU oracle for the few-mismatch search phase -- test infrastructure only.
 *
 * The paper's first phase aligns each read with few mismatches through a BWT
 * index of the reference and hands the reads it cannot place to DP (Methods,
 * architecture & parallelism; extra parallelism: the BWT queries are the
 * other bottleneck).  The index is a means; what the phase computes has a
 * plain definition, and this file is that definition written out:
 *
 *   hits(read) = { p : 0 <= p <= L - m, Hamming(read, ref[p, p + m)) <= k }
 *
 * for a read of m bases, a reference of L bases (forward strand, one
 * sequence) and 0 <= k <= 2.  Per read it reports the smallest mismatch
 * count over the hits (-1 without hits), how many hits have it, how many
 * hits there are, and the leftmost hit with the smallest count.
 *
 * Readings (the paper gives none of these):
 *  - the read is cut into k + 1 parts, part j = [floor(j m / (k+1)),
 *    floor((j+1) m / (k+1))); a read is repetitive when some part occurs
 *    exactly more than max_occ times anywhere in the reference (its
 *    occurrences counted over all q in [0, L - len]).  A repetitive read is
 *    not searched: status REPETITIVE, best -1, counts 0, position -1.  This
 *    stands for the paper's threads leaving resource-demanding repetitive
 *    reads to the host.
 *  - m < k + 1 (an empty part) or m > MAX_M is a length error.
 *
 * Everything is brute force over every reference position, one read per task
 * on a pthread pool.  It shares no code with the GPU library.
 */
#include <pthread.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#define KMM_MAX_M 1024
#define KMM_ST_LEN_LIMIT (1u << 2)
#define KMM_ST_READ_OOB (1u << 4)
#define KMM_ST_REPETITIVE (1u << 6)

typedef struct {
  const uint8_t *ref;
  int64_t ref_len;
  const uint8_t *reads;
  int64_t reads_len;
  const int64_t *read_off;
  const int32_t *read_len;
  int64_t n_reads;
  int32_t k, max_occ;
  int32_t *best_mm, *n_best, *n_hits;
  int64_t *pos;
  uint32_t *status;
  int64_t next;
  pthread_mutex_t lock;
} kmm_job_t;

/* exact occurrences of s[0, len) in ref, counted up to limit + 1 */
static int64_t count_exact(const uint8_t *ref, int64_t L, const uint8_t *s, int32_t len, int64_t limit) {
  int64_t c = 0;
  for (int64_t q = 0; q + len <= L; q++) {
    int32_t t = 0;
    while (t < len && ref[q + t] == s[t]) t++;
    if (t == len && ++c > limit) break;
  }
  return c;
}

static void search_one(kmm_job_t *J, int64_t r) {
  const int32_t m = J->read_len[r];
  const int32_t k = J->k;
  J->best_mm[r] = -1;
  J->n_best[r] = 0;
  J->n_hits[r] = 0;
  J->pos[r] = -1;
  J->status[r] = 0;
  if (m < k + 1 || m > KMM_MAX_M) {
    J->status[r] = KMM_ST_LEN_LIMIT;
    return;
  }
  if (J->read_off[r] < 0 || J->read_off[r] + m > J->reads_len) {
    J->status[r] = KMM_ST_READ_OOB;
    return;
  }
  const uint8_t *q = J->reads + J->read_off[r];
  /* the repetitive rule: exact occurrences of each of the k + 1 parts */
  for (int32_t j = 0; j <= k; j++) {
    const int32_t a = (int32_t)((int64_t)j * m / (k + 1));
    const int32_t b = (int32_t)((int64_t)(j + 1) * m / (k + 1));
    if (count_exact(J->ref, J->ref_len, q + a, b - a, J->max_occ) > J->max_occ) {
      J->status[r] = KMM_ST_REPETITIVE;
      return;
    }
  }
  /* the definition: every placement of the whole read */
  int32_t best = -1, nb = 0, nh = 0;
  int64_t bp = -1;
  for (int64_t p = 0; p + m <= J->ref_len; p++) {
    int32_t d = 0;
    for (int32_t t = 0; t < m && d <= k; t++) d += J->ref[p + t] != q[t];
    if (d > k) continue;
    nh++;
    if (best < 0 || d < best) {
      best = d;
      nb = 1;
      bp = p;
    } else if (d == best) {
      nb++;
    }
  }
  J->best_mm[r] = best;
  J->n_best[r] = nb;
  J->n_hits[r] = nh;
  J->pos[r] = bp;
}

static void *kmm_worker(void *arg) {
  kmm_job_t *J = (kmm_job_t *)arg;
  for (;;) {
    pthread_mutex_lock(&J->lock);
    const int64_t r = J->next++;
    pthread_mutex_unlock(&J->lock);
    if (r >= J->n_reads) break;
    search_one(J, r);
  }
  return NULL;
}

/* Search n_reads reads (one base code per byte, A0 C1 G2 T3) against ref.
 * Returns 0, or -1 when k is outside 0..2 or max_occ < 1. */
int oracle_kmm_search(const uint8_t *ref, int64_t ref_len, const uint8_t *reads, int64_t reads_len,
                      const int64_t *read_off, const int32_t *read_len, int64_t n_reads, int32_t k,
                      int32_t max_occ, int32_t *best_mm, int32_t *n_best, int32_t *n_hits, int64_t *pos,
                      uint32_t *status, int32_t n_threads) {
  if (k < 0 || k > 2 || max_occ < 1 || n_reads < 0) return -1;
  kmm_job_t J;
  memset(&J, 0, sizeof(J));
  J.ref = ref;
  J.ref_len = ref_len;
  J.reads = reads;
  J.reads_len = reads_len;
  J.read_off = read_off;
  J.read_len = read_len;
  J.n_reads = n_reads;
  J.k = k;
  J.max_occ = max_occ;
  J.best_mm = best_mm;
  J.n_best = n_best;
  J.n_hits = n_hits;
  J.pos = pos;
  J.status = status;
  pthread_mutex_init(&J.lock, NULL);
  if (n_threads < 1) n_threads = 1;
  if (n_threads > 256) n_threads = 256;
  pthread_t th[256];
  for (int t = 0; t < n_threads; t++) pthread_create(&th[t], NULL, kmm_worker, &J);
  for (int t = 0; t < n_threads; t++) pthread_join(th[t], NULL);
  pthread_mutex_destroy(&J.lock);
  return 0;
}
