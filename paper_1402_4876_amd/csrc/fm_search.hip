// Few-mismatch search: exact backward search of the read's k + 1 parts in the
// FM index, occurrences from the suffix array, verification of every
// candidate placement on the 2-bit reference (pigeonhole: a placement with
// at most k mismatches has an exact part).
#include <hip/hip_runtime.h>

#include "ctx.h"
#include "fm_common.h"
#include "fm_match.h"
#include "mica_fm.h"

namespace mica {
namespace {

constexpr int kLanesPerRead = 4;  // lane j searches part j (k + 1 <= 3 parts)

struct FmSearchArgs {
  FmIndex ix;
  const uint32_t* reads2b;
  uint64_t reads_len;
  uint64_t read_words;
  const uint64_t* read_off;
  const int32_t* read_len;
  int64_t n_reads;
  int32_t k, max_occ;
  int32_t *best_mm, *n_best, *n_hits;
  int64_t* pos;
  uint32_t* status;
  int64_t* cand;
};

using fm::base_at;
using fm::diff_mask;

// Occ(c, i): occurrences of base c in BWT rows [0, i)
__device__ __forceinline__ uint32_t occ(const FmIndex& ix, uint32_t c, uint32_t i) {
  const uint32_t b = i / kFmBlockSyms, o = i - b * kFmBlockSyms;
  const uint4* blk = (const uint4*)(ix.occ + (size_t)b * kFmBlockWords);
  const uint4 h = blk[0];
  uint32_t w[12];
  const uint4 q0 = blk[1], q1 = blk[2], q2 = blk[3];
  w[0] = q0.x; w[1] = q0.y; w[2] = q0.z; w[3] = q0.w;
  w[4] = q1.x; w[5] = q1.y; w[6] = q1.z; w[7] = q1.w;
  w[8] = q2.x; w[9] = q2.y; w[10] = q2.z; w[11] = q2.w;
  uint32_t n = c == 0 ? h.x : (c == 1 ? h.y : (c == 2 ? h.z : h.w));
  const uint32_t pat = c * 0x55555555u;
  const uint32_t full = o >> 4, part = o & 15;
#pragma unroll
  for (uint32_t t = 0; t < 12; ++t) {
    const uint32_t match = ~diff_mask(w[t], pat) & 0x55555555u;
    const uint32_t keep = t < full ? 0x55555555u : (t == full ? (1u << (2 * part)) - 1u : 0u);
    n += __popc(match & keep);
  }
  // the sentinel row holds code 0 but is no base
  if (c == 0 && ix.dollar >= b * kFmBlockSyms && ix.dollar < i) n -= 1;
  return n;
}

__global__ __launch_bounds__(256) void k_fm_search(FmSearchArgs A) {
  const int64_t gid = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const int64_t r = gid / kLanesPerRead;
  const int j = (int)(gid % kLanesPerRead);
  const bool live = r < A.n_reads;
  const int k = A.k;
  int m = 0;
  uint64_t ro = 0;
  uint32_t st = 0;
  if (live) {
    m = A.read_len[r];
    ro = A.read_off[r];
    if (m < k + 1 || m > MICA_MAX_READ_LEN) st = MICA_ST_LEN_LIMIT;
    else if (ro > A.reads_len || (uint64_t)m > A.reads_len - ro) st = MICA_ST_READ_OOB;
  }
  const fm::Stretch S{A.reads2b, A.read_words, A.ix.ref2b, A.ix.ref_words};
  int rep = 0, best = 0x7FFFFFFF, nb = 0, nh = 0;
  int64_t bp = 0x7FFFFFFFFFFFFFFFll;
  if (live && st == 0 && j <= k) {
    const int a = (int)((int64_t)j * m / (k + 1));
    const int e = (int)((int64_t)(j + 1) * m / (k + 1));
    // exact backward search of part j, its last base first
    uint32_t lo = 0, hi = (uint32_t)(A.ix.n + 1);
    for (int t = e - 1; t >= a && lo < hi; --t) {
      const uint32_t c = base_at(A.reads2b, ro + (uint64_t)t);
      lo = A.ix.C[c] + occ(A.ix, c, lo);
      hi = A.ix.C[c] + occ(A.ix, c, hi);
    }
    if (lo < hi && hi - lo > (uint32_t)A.max_occ) {
      rep = 1;
    } else {
      int64_t seed = MICA_FM_NO_CAND;
      for (uint32_t i = lo; i < hi; ++i) {
        const int64_t p = (int64_t)A.ix.sa[i] - a;
        seed = (seed == MICA_FM_NO_CAND || p < seed) ? p : seed;
        if (p < 0 || (uint64_t)p + (uint64_t)m > A.ix.n) continue;
        // counted by the lowest-index exact part only (parts 0 and 1 are the
        // only ones below another part, k <= 2)
        bool mine = true;
        if (j >= 1) {
          const int e0 = (int)((int64_t)m / (k + 1));
          mine = !fm::exact(S, ro, (uint64_t)p, e0);
        }
        if (j >= 2 && mine) {
          const int a1 = (int)((int64_t)m / (k + 1));
          const int e1 = (int)((int64_t)2 * m / (k + 1));
          mine = !fm::exact(S, ro + a1, (uint64_t)p + a1, e1 - a1);
        }
        if (!mine) continue;
        const int d = fm::mismatches(S, ro, (uint64_t)p, m, k);
        if (d > k) continue;
        ++nh;
        if (d < best) {
          best = d;
          nb = 1;
          bp = p;
        } else if (d == best) {
          ++nb;
          bp = p < bp ? p : bp;
        }
      }
      if (A.cand) A.cand[r * 3 + j] = seed;
    }
  }
  if (A.cand && live && j < 3 && (st != 0 || j > k || rep)) A.cand[r * 3 + j] = MICA_FM_NO_CAND;
  // the read's four lanes combine their hits
#pragma unroll
  for (int x = 1; x < kLanesPerRead; x <<= 1) {
    rep |= __shfl_xor(rep, x, kLanesPerRead);
    const int ob = __shfl_xor(best, x, kLanesPerRead);
    const int onb = __shfl_xor(nb, x, kLanesPerRead);
    const int64_t obp = __shfl_xor(bp, x, kLanesPerRead);
    nh += __shfl_xor(nh, x, kLanesPerRead);
    if (ob < best) {
      best = ob;
      nb = onb;
      bp = obp;
    } else if (ob == best) {
      nb += onb;
      bp = obp < bp ? obp : bp;
    }
  }
  if (live && j == 0) {
    if (st == 0 && rep) st = MICA_ST_REPETITIVE;
    const bool found = st == 0 && best <= k;
    A.best_mm[r] = found ? best : -1;
    A.n_best[r] = found ? nb : 0;
    A.n_hits[r] = st == 0 ? nh : 0;
    A.pos[r] = found ? bp : -1;
    A.status[r] = st;
  }
}

}  // namespace
}  // namespace mica

extern "C" mica_status_t mica_fm_search(mica_fm_t f, const mica_fm_batch_t* b, void* stream) {
  using namespace mica;
  if (!f || !b) return fail(MICA_ERR_INVALID_ARG, "NULL index or batch");
  if (b->k < 0 || b->k > 2) return fail(MICA_ERR_INVALID_ARG, "k must be 0, 1 or 2");
  if (b->max_occ < 1 || b->max_occ > MICA_FM_MAX_OCC) return fail(MICA_ERR_INVALID_ARG, "max_occ outside 1..65536");
  if (b->n_reads < 0) return fail(MICA_ERR_INVALID_ARG, "negative n_reads");
  if (b->n_reads == 0) return MICA_OK;
  if (!b->reads2b || !b->read_off || !b->read_len || !b->best_mm || !b->n_best || !b->n_hits || !b->pos ||
      !b->status)
    return fail(MICA_ERR_INVALID_ARG, "NULL batch array");
  FmSearchArgs A;
  A.ix = *fm_index_of(f);
  A.reads2b = b->reads2b;
  A.reads_len = b->reads_len;
  A.read_words = (b->reads_len + 15) / 16;
  A.read_off = b->read_off;
  A.read_len = b->read_len;
  A.n_reads = b->n_reads;
  A.k = b->k;
  A.max_occ = b->max_occ;
  A.best_mm = b->best_mm;
  A.n_best = b->n_best;
  A.n_hits = b->n_hits;
  A.pos = b->pos;
  A.status = b->status;
  A.cand = b->cand;
  const int64_t threads = b->n_reads * kLanesPerRead;
  const int64_t blocks = (threads + 255) / 256;
  if (blocks > 0x7FFFFFFF) return fail(MICA_ERR_LIMIT, "too many reads for one launch");
  HIP_TRY(hipSetDevice(A.ix.device));
  hipLaunchKernelGGL(k_fm_search, dim3((unsigned)blocks), dim3(256), 0, (hipStream_t)stream, A);
  HIP_TRY(hipGetLastError());
  return MICA_OK;
}
