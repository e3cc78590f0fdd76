/*
 * Reference oracle for affine-gap (Gotoh) read alignment -- TEST INFRASTRUCTURE.
 *
 * This file is a plain, slow, full-matrix CPU implementation of what the
 * GPU library computes.  Only the test-suite, the smoke check and the
 * benchmark's CPU baseline may load it.  It shares no code, header, table
 * or helper with the HIP library, and the library never calls it.
 *
 * What it follows (MICA, "Highly parallel dynamic programming"):
 *   - the DP table T over read rows i and region columns j, where cell (i,j)
 *     depends on its upper, upper-left and left neighbours;
 *   - the affine gap model with three tables, one for alignments ending in
 *     a Match (here the diagonal candidate M = H(i-1,j-1)+s), one ending in
 *     an Insert (I, consumes a read base only) and one ending in a Delete
 *     (D, consumes a reference base only); H(i,j) = max(M, I, D);
 *   - the method turns to DP for reads that need gaps or clipped ends
 *     (Methods, architecture section and DP section), hence two modes: semi-global
 *     (whole read against any substring of the window) and local
 *     (Smith-Waterman, both ends free: the clipped ends).
 *   - the extension mode (mode 2) is the read-extension use of DP with
 *     clipping: the alignment is anchored at (0,0) with a start score h0 (the
 *     score of the exact seed it extends), and the read may end early
 *     (clipped) unless aligning it to its end scores within a clipping
 *     penalty of the best early end.
 * The paper gives no scores, boundaries, tie-breaks, or CIGAR rules; the
 * readings used here are stated next to each step and listed in the design
 * notes.  Everything is exact int32 arithmetic: every reachable value is far
 * from the NEG sentinel for the supported limits (m <= 1024, n <= 8192,
 * |score parameters| <= 4096).
 *
 * Parity status: pinned.  The CPU tests check this file against exhaustive
 * enumeration of all alignments of small sequences (score, end cell and the
 * canonical traceback), against closed forms and against invariants.
 */
#include <pthread.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#define ORA_NEG (-(1 << 30))

/* per-pair status bits (same meaning as the library's status word) */
#define ORA_ST_CIGAR_TRUNC (1u << 1)
#define ORA_ST_LEN_LIMIT (1u << 2)
#define ORA_ST_WIN_OOB (1u << 3)
#define ORA_ST_READ_OOB (1u << 4)

#define ORA_MAX_M 1024
#define ORA_MAX_H0 (1 << 20)
#define ORA_MAX_N 8192

/* CIGAR op codes as in BAM: M=0, I=1, D=2; a CIGAR word is len<<4 | op */
enum { OP_M = 0, OP_I = 1, OP_D = 2 };

typedef struct {
  /* inputs: one base code (A0 C1 G2 T3) per byte */
  const uint8_t *ref;
  int64_t ref_len;
  const int64_t *win_off;
  const int32_t *win_len;
  const uint8_t *reads;
  int64_t reads_len;
  const int64_t *read_off;
  const int32_t *read_len;
  const uint8_t *mode; /* 0 = semi-global, 1 = local, 2 = extension; NULL: default_mode */
  int32_t default_mode;
  const int32_t *h0;   /* extension start score per pair; NULL: default_h0 */
  int32_t default_h0;
  int32_t clip;        /* extension clipping penalty */
  int64_t n_pairs;
  int32_t a, b, o, e; /* match, mismatch, gap open, gap extend */
  int32_t want_trace; /* compute starts and CIGAR */
  int32_t cigar_cap;
  /* outputs */
  int32_t *score, *read_start, *read_end, *ref_start, *ref_end;
  uint32_t *cigar;
  int32_t *n_cigar;
  uint32_t *status;
  /* work distribution */
  int64_t next;
  pthread_mutex_t lock;
} ora_job_t;

typedef struct {
  int32_t *H, *D, *I;
  size_t cap; /* cells */
  uint8_t *ops; /* reversed op list, one byte per emitted op */
  size_t ops_cap;
} ora_ws_t;

static int ws_reserve(ora_ws_t *w, size_t cells, size_t nops) {
  if (cells > w->cap) {
    free(w->H);
    free(w->D);
    free(w->I);
    w->H = (int32_t *)malloc(cells * sizeof(int32_t));
    w->D = (int32_t *)malloc(cells * sizeof(int32_t));
    w->I = (int32_t *)malloc(cells * sizeof(int32_t));
    if (!w->H || !w->D || !w->I) return -1;
    w->cap = cells;
  }
  if (nops > w->ops_cap) {
    free(w->ops);
    w->ops = (uint8_t *)malloc(nops);
    if (!w->ops) return -1;
    w->ops_cap = nops;
  }
  return 0;
}

static inline int32_t imax(int32_t x, int32_t y) { return x > y ? x : y; }

/* Align read q[0..m) against window r[0..n) in mode md (0 semi-global,
 * 1 local, 2 extension with start score h0) and write the outputs of pair p. */
static void align_one(ora_job_t *J, ora_ws_t *W, int64_t p, const uint8_t *q, int m,
                      const uint8_t *r, int n, int md, int32_t h0) {
  const int32_t a = J->a, b = J->b, o = J->o, e = J->e;
  const int local = md == 1, ext = md == 2;
  const int W1 = n + 1; /* row stride */
  int32_t *H = W->H, *D = W->D, *I = W->I;
#define AT(X, i, j) X[(size_t)(i) * W1 + (j)]

  /* Boundaries.
   * Semi-global: the read is aligned end to end, the window is free at both
   * ends: H(0,j) = 0 for every j; H(i,0) = I(i,0) = -(o + i*e) (a leading
   * insertion before the window); D(i,0) = NEG; D(0,j) = I(0,j) = NEG.
   * Local: H(0,j) = H(i,0) = 0; D and I are NEG on row 0 and column 0.
   * Extension: anchored at (0,0) with score h0: H(0,0) = h0; a leading
   * deletion H(0,j) = D(0,j) = h0 - (o + j*e), I(0,j) = NEG; a leading
   * insertion H(i,0) = I(i,0) = h0 - (o + i*e), D(i,0) = NEG. */
  for (int j = 0; j <= n; j++) {
    AT(H, 0, j) = ext ? (j == 0 ? h0 : h0 - (o + j * e)) : 0;
    AT(D, 0, j) = (ext && j > 0) ? h0 - (o + j * e) : ORA_NEG;
    AT(I, 0, j) = ORA_NEG;
  }
  for (int i = 1; i <= m; i++) {
    AT(H, i, 0) = local ? 0 : (ext ? h0 : 0) - (o + i * e);
    AT(I, i, 0) = local ? ORA_NEG : (ext ? h0 : 0) - (o + i * e);
    AT(D, i, 0) = ORA_NEG;
  }

  /* Recurrences (affine gaps; a gap of length L scores -(o + L*e)):
   *   D(i,j) = max(D(i,j-1) - e, H(i,j-1) - o - e)    deletion, horizontal
   *   I(i,j) = max(I(i-1,j) - e, H(i-1,j) - o - e)    insertion, vertical
   *   H(i,j) = max(H(i-1,j-1) + s(q_i, r_j), D(i,j), I(i,j)) [, 0 if local]
   * filled row by row: each cell only needs its left, upper and upper-left
   * neighbours. */
  for (int i = 1; i <= m; i++) {
    const int qi = q[i - 1];
    for (int j = 1; j <= n; j++) {
      const int32_t s = (qi == r[j - 1]) ? a : b;
      const int32_t d = imax(AT(D, i, j - 1) - e, AT(H, i, j - 1) - o - e);
      const int32_t ins = imax(AT(I, i - 1, j) - e, AT(H, i - 1, j) - o - e);
      int32_t h = imax(AT(H, i - 1, j - 1) + s, imax(d, ins));
      if (local) h = imax(h, 0);
      AT(D, i, j) = d;
      AT(I, i, j) = ins;
      AT(H, i, j) = h;
    }
  }

  /* Result cell.  Semi-global: row m, the largest H(m,j) over j in [0,n],
   * ties to the smallest j.  Local: the largest H over (0,0) (value 0) and
   * every cell with i,j >= 1, ties to the smallest j, then the smallest i.
   * Scanning j outer / i inner and replacing only on a strictly larger
   * value realises exactly that order.
   * Extension: the best early end is the local rule with (0,0) worth h0;
   * the best end-to-end end is the semi-global rule on row m; the read is
   * aligned to its end when that scores at least the early end minus the
   * clipping penalty, and clipped otherwise. */
  int bi = 0, bj = 0;
  int32_t best;
  if (md == 0) {
    bi = m;
    best = AT(H, m, 0);
    for (int j = 1; j <= n; j++)
      if (AT(H, m, j) > best) {
        best = AT(H, m, j);
        bj = j;
      }
  } else {
    best = ext ? h0 : 0;
    for (int j = 1; j <= n; j++)
      for (int i = 1; i <= m; i++)
        if (AT(H, i, j) > best) {
          best = AT(H, i, j);
          bi = i;
          bj = j;
        }
    if (ext) {
      int32_t gbest = AT(H, m, 0);
      int gj = 0;
      for (int j = 1; j <= n; j++)
        if (AT(H, m, j) > gbest) {
          gbest = AT(H, m, j);
          gj = j;
        }
      if ((int64_t)gbest >= (int64_t)best - J->clip) {
        best = gbest;
        bi = m;
        bj = gj;
      }
    }
  }
  J->score[p] = best;
  J->read_end[p] = bi;
  J->ref_end[p] = bj;
  if (!J->want_trace) return;

  /* Traceback from (bi, bj) in state H with priorities
   *   zero (local) > diagonal > D > I, and gap open > gap extend,
   * decided by equality tests on the stored matrices.  An extension ends at
   * the anchor (0,0): on row 0 the rest is a leading deletion, on column 0
   * a leading insertion. */
  enum { ST_H, ST_D, ST_I } st = ST_H;
  int i = bi, j = bj;
  size_t nops = 0;
  uint8_t *ops = W->ops;
  for (;;) {
    if (st == ST_H) {
      if (local && AT(H, i, j) == 0) break;
      if (ext && i == 0) {
        for (; j > 0; j--) ops[nops++] = OP_D;
        break;
      }
      if (i == 0) break;
      if (!local && j == 0) {
        for (; i > 0; i--) ops[nops++] = OP_I;
        break;
      }
      const int32_t s = (q[i - 1] == r[j - 1]) ? a : b;
      if (AT(H, i, j) == AT(H, i - 1, j - 1) + s) {
        ops[nops++] = OP_M;
        i--;
        j--;
      } else if (AT(H, i, j) == AT(D, i, j)) {
        st = ST_D;
      } else {
        st = ST_I;
      }
    } else if (st == ST_D) {
      ops[nops++] = OP_D;
      if (AT(D, i, j) == AT(H, i, j - 1) - o - e) st = ST_H;
      j--;
    } else {
      ops[nops++] = OP_I;
      if (AT(I, i, j) == AT(H, i - 1, j) - o - e) st = ST_H;
      i--;
    }
  }
  J->read_start[p] = i;
  J->ref_start[p] = j;
#undef AT

  /* ops[] is in reverse order; emit run-length words front to back. */
  int32_t nrun = 0;
  const int32_t cap = J->cigar_cap;
  uint32_t *cg = J->cigar ? J->cigar + (size_t)p * (size_t)(cap > 0 ? cap : 0) : NULL;
  size_t k = nops;
  while (k > 0) {
    const uint8_t op = ops[k - 1];
    uint32_t len = 0;
    while (k > 0 && ops[k - 1] == op) {
      len++;
      k--;
    }
    if (cg && nrun < cap) cg[nrun] = (len << 4) | op;
    nrun++;
  }
  if (nrun > cap) {
    J->status[p] |= ORA_ST_CIGAR_TRUNC;
    J->n_cigar[p] = -nrun;
  } else {
    J->n_cigar[p] = nrun;
  }
}

static void run_pair(ora_job_t *J, ora_ws_t *W, int64_t p) {
  const int32_t m = J->read_len[p], n = J->win_len[p];
  const int md = J->mode ? J->mode[p] : J->default_mode;
  const int32_t h0 = J->h0 ? J->h0[p] : J->default_h0;
  J->status[p] = 0;
  J->score[p] = 0;
  J->read_end[p] = 0;
  J->ref_end[p] = 0;
  if (J->want_trace) {
    J->read_start[p] = 0;
    J->ref_start[p] = 0;
    J->n_cigar[p] = 0;
  }
  if (m < 0 || n < 0 || m > ORA_MAX_M || n > ORA_MAX_N || md < 0 || md > 2 || (md == 2 && (h0 < 0 || h0 > ORA_MAX_H0))) {
    J->status[p] = ORA_ST_LEN_LIMIT;
    return;
  }
  if (J->win_off[p] < 0 || J->win_off[p] + n > J->ref_len) {
    J->status[p] = ORA_ST_WIN_OOB;
    return;
  }
  if (J->read_off[p] < 0 || J->read_off[p] + m > J->reads_len) {
    J->status[p] = ORA_ST_READ_OOB;
    return;
  }
  if (ws_reserve(W, (size_t)(m + 1) * (size_t)(n + 1), (size_t)(m + n + 1)) != 0) abort();
  align_one(J, W, p, J->reads + J->read_off[p], m, J->ref + J->win_off[p], n, md, h0);
}

static void *worker(void *arg) {
  ora_job_t *J = (ora_job_t *)arg;
  ora_ws_t W;
  memset(&W, 0, sizeof(W));
  const int64_t chunk = 256;
  for (;;) {
    pthread_mutex_lock(&J->lock);
    int64_t lo = J->next;
    J->next += chunk;
    pthread_mutex_unlock(&J->lock);
    if (lo >= J->n_pairs) break;
    int64_t hi = lo + chunk < J->n_pairs ? lo + chunk : J->n_pairs;
    for (int64_t p = lo; p < hi; p++) run_pair(J, &W, p);
  }
  free(W.H);
  free(W.D);
  free(W.I);
  free(W.ops);
  return NULL;
}

/* Align n_pairs pairs on n_threads host threads (dynamic chunks of 256
 * pairs).  Sequences are one code per byte.  Returns 0, or -1 on invalid
 * scoring.  read_start, ref_start, cigar and n_cigar are used only when
 * want_trace is non-zero; cigar holds cigar_cap words per pair.  Extension
 * pairs (mode 2) take their start score from h0[p] (h0 NULL: default_h0)
 * and the clipping penalty clip. */
int oracle_align_batch_ext(const uint8_t *ref, int64_t ref_len, const int64_t *win_off,
                           const int32_t *win_len, const uint8_t *reads, int64_t reads_len,
                           const int64_t *read_off, const int32_t *read_len, const uint8_t *mode,
                           int32_t default_mode, const int32_t *h0, int32_t default_h0, int32_t clip,
                           int64_t n_pairs, int32_t match, int32_t mismatch, int32_t gap_open,
                           int32_t gap_extend, int32_t want_trace, int32_t cigar_cap, int32_t *score,
                           int32_t *read_start, int32_t *read_end, int32_t *ref_start, int32_t *ref_end,
                           uint32_t *cigar, int32_t *n_cigar, uint32_t *status, int32_t n_threads) {
  if (match < 1 || match > 4096 || mismatch > 0 || mismatch < -4096 || gap_open < 0 ||
      gap_open > 4096 || gap_extend < 1 || gap_extend > 4096)
    return -1;
  if (n_pairs < 0 || cigar_cap < 0 || clip < 0 || clip > ORA_MAX_H0) return -1;
  ora_job_t J;
  memset(&J, 0, sizeof(J));
  J.ref = ref;
  J.ref_len = ref_len;
  J.win_off = win_off;
  J.win_len = win_len;
  J.reads = reads;
  J.reads_len = reads_len;
  J.read_off = read_off;
  J.read_len = read_len;
  J.mode = mode;
  J.default_mode = default_mode;
  J.h0 = h0;
  J.default_h0 = default_h0;
  J.clip = clip;
  J.n_pairs = n_pairs;
  J.a = match;
  J.b = mismatch;
  J.o = gap_open;
  J.e = gap_extend;
  J.want_trace = want_trace;
  J.cigar_cap = cigar_cap;
  J.score = score;
  J.read_start = read_start;
  J.read_end = read_end;
  J.ref_start = ref_start;
  J.ref_end = ref_end;
  J.cigar = cigar;
  J.n_cigar = n_cigar;
  J.status = status;
  J.next = 0;
  pthread_mutex_init(&J.lock, NULL);
  if (n_threads < 1) n_threads = 1;
  if (n_threads == 1) {
    worker(&J);
  } else {
    pthread_t *th = (pthread_t *)malloc(sizeof(pthread_t) * (size_t)n_threads);
    for (int t = 0; t < n_threads; t++) pthread_create(&th[t], NULL, worker, &J);
    for (int t = 0; t < n_threads; t++) pthread_join(th[t], NULL);
    free(th);
  }
  pthread_mutex_destroy(&J.lock);
  return 0;
}

/* The semi-global / local entry point (no extension parameters). */
int oracle_align_batch(const uint8_t *ref, int64_t ref_len, const int64_t *win_off,
                       const int32_t *win_len, const uint8_t *reads, int64_t reads_len,
                       const int64_t *read_off, const int32_t *read_len, const uint8_t *mode,
                       int32_t default_mode, int64_t n_pairs, int32_t match, int32_t mismatch,
                       int32_t gap_open, int32_t gap_extend, int32_t want_trace,
                       int32_t cigar_cap, int32_t *score, int32_t *read_start,
                       int32_t *read_end, int32_t *ref_start, int32_t *ref_end, uint32_t *cigar,
                       int32_t *n_cigar, uint32_t *status, int32_t n_threads) {
  return oracle_align_batch_ext(ref, ref_len, win_off, win_len, reads, reads_len, read_off, read_len, mode,
                                default_mode, NULL, 0, 0, n_pairs, match, mismatch, gap_open, gap_extend,
                                want_trace, cigar_cap, score, read_start, read_end, ref_start, ref_end,
                                cigar, n_cigar, status, n_threads);
}
