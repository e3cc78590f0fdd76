// Planning, bucketing, 2-bit packing and saturated-pair re-run kernels, and
// the table of kernel entry points used by the host runtime.
#include "dp_fill.h"
#include "plan.h"

namespace mica {

// Exact 32-bit recomputation of the pairs whose 16-bit scores saturated.
template <bool DIR>
__global__ __launch_bounds__(256) void k_rerun(const Params* __restrict__ prm) {
  extern __shared__ uint32_t smem[];
  const int wave = uni((int)(threadIdx.x >> 6));
  const int slot_id = blockIdx.x * kWavesPerBlock + wave;
  if (slot_id >= prm->n_slots) return;
  uint32_t* lds = smem + wave * kLdsWaveWords;
  uint8_t* slot = prm->scratch + (size_t)slot_id * prm->slot_bytes;
  const uint32_t cnt = prm->counters[kCtrRerun];
  const uint32_t n_waves = gridDim.x * (uint32_t)kWavesPerBlock;
  for (uint32_t it = (uint32_t)slot_id; it < cnt; it += n_waves) {
    const uint32_t* pp = prm->rerun + it;
    const int p = (int)*pp;
    const int md = prm->mode ? prm->mode[p] : prm->default_mode;
    // a full traceback: the re-run is rare and needs no band
    constexpr int TB = DIR ? kTbFull : kTbNone;
    if (md == 2) process_item<V32, 64, 16, 2, TB, false>(prm, pp, 1, lds, slot, -1);
    else if (md == 1) process_item<V32, 64, 16, 1, TB, false>(prm, pp, 1, lds, slot, -1);
    else process_item<V32, 64, 16, 0, TB, false>(prm, pp, 1, lds, slot, -1);
    if ((threadIdx.x & 63) == 0) prm->status[p] |= kStSaturated;
  }
}

// ----------------------------------------------------------------------------
// planning: validation, trivial pairs, bucket histogram, work queue

__global__ void k_zero(const Params* __restrict__ prm) {
  for (int i = threadIdx.x; i < kNumSubBuckets; i += blockDim.x) prm->scount[i] = 0;
  const int i = threadIdx.x;
  if (i < kNumBuckets) {
    prm->bhead[i] = 0;
    prm->fbcount[i] = 0;
    prm->dbcount[i] = 0;
    prm->dbwide[i] = 0;
    prm->sidehead[i] = 0;
  }
  if (i < kNumCounters) prm->counters[i] = 0;
}

// Can every value of the pair's DP stay inside int16 (with a guard band)?
// Semi-global and local values are shifted by -d0 (dummy rows above the
// read).  An extension starts from h0: no cell exceeds h0 + a min(m, n),
// and every cell is at least what the path of j deletions along row 0 and i
// insertions down column j gives, h0 - 2o - (i + j)e, so every H, gap and
// boundary value is at least h0 - 3o - (m + n + 1)e.  (Rows below the read
// only feed rows further below; their values may clamp.)
__device__ __forceinline__ bool int16_safe(int m, int n, int mode, int d0, int a, int b, int o, int e, int h0) {
  long hi, lo;
  if (mode == 2) {
    hi = (long)h0 + (long)a * (long)(m < n ? m : n);
    lo = (long)h0 - 3L * o - (long)(m + n + 1) * e;
  } else {
    hi = (long)a * (long)(m < n ? m : n) - d0;
    lo = (mode ? -(long)(o + e) : -(long)(2 * o + (long)(m + 1) * e)) - d0;
  }
  (void)b;
  return hi <= 32767 - 8 && lo >= -32767 + 8;
}

__global__ __launch_bounds__(kPlanThreads) void k_plan(const Params* __restrict__ prm) {
  __shared__ uint32_t hist[kNumSubBuckets];
  for (int i = threadIdx.x; i < kNumSubBuckets; i += blockDim.x) hist[i] = 0;
  __syncthreads();
  for (int rep = 0; rep < kPlanPairsPerThread; ++rep) {
    const int64_t p = ((int64_t)blockIdx.x * kPlanPairsPerThread + rep) * blockDim.x + threadIdx.x;
    if (p < prm->n_pairs) {
      const int m = prm->read_len[p], n = prm->win_len[p];
      const int md = prm->mode ? (int)prm->mode[p] : prm->default_mode;
      const uint64_t wo = prm->win_off[p], ro = prm->read_off[p];
      const int h0 = md == 2 ? (prm->ext_h0 ? prm->ext_h0[p] : prm->ext_default_h0) : 0;
      uint32_t st = 0;
      if (m < prm->min_m || n < 0 || m > prm->max_m || n > prm->max_n || md < 0 || md > 2 || !((prm->mode_mask >> md) & 1) ||
          h0 < 0 || h0 > prm->max_h0)
        st = kStLenLimit;
      else if (wo > prm->ref_len || (uint64_t)n > prm->ref_len - wo) st = kStWinOob;
      else if (ro > prm->reads_len || (uint64_t)m > prm->reads_len - ro) st = kStReadOob;
      const bool want_start = (prm->flags & (kOutStart | kOutCigar)) != 0;
      const bool want_cigar = (prm->flags & kOutCigar) != 0;
      uint32_t b = kSkip;
      if (st != 0 || m == 0 || n == 0) {
        int score = 0, re = 0;
        int ncig = 0;
        // semi-global against an empty window: all insertions; an extension
        // with an empty read or window: the anchor itself, or (empty window)
        // all insertions when that is within the clipping penalty
        const bool all_ins = st == 0 && m > 0 &&
                             (md == 0 || (md == 2 && (long)prm->so + (long)m * prm->se <= (long)prm->ext_clip));
        if (st == 0 && md == 2) score = h0;
        if (all_ins) {
          score = (md == 2 ? h0 : 0) - (prm->so + m * prm->se);
          re = m;
          ncig = 1;
          if (want_cigar) {
            if (prm->cigar_cap >= 1) prm->cigar[(size_t)p * prm->cigar_cap] = ((uint32_t)m << 4) | 1u;
            else st |= kStCigarTrunc;
          }
        }
        prm->score[p] = score;
        prm->read_end[p] = re;
        prm->ref_end[p] = 0;
        if (want_start) {
          prm->read_start[p] = 0;
          prm->ref_start[p] = 0;
        }
        if (want_cigar) prm->n_cigar[p] = (st & kStCigarTrunc) ? -ncig : ncig;
        prm->status[p] = st;
      } else {
        const int cls = prm->class_of_m[m];
        const int d0 = class_lanes(cls) * class_rows(cls) - m;
        // the 16-bit bounds hold for the fallback class's dummy rows too
        // (at least as many as the pair's own class)
        const int fbc = fallback_class(cls);
        const int d0k = class_lanes(fbc) * class_rows(fbc) - m;
        int kind;
        if (prm->flags & kForceInt32) kind = kK32;
        else kind = int16_safe(m, n, md, d0k, prm->sa, prm->sb, prm->so, prm->se, h0) ? kK16 : kK16Sat;
        b = (uint32_t)(bucket_id(kind, cls, md) * kSubBins + sub_bin(cls, d0));
        atomicAdd(&hist[b], 1u);
      }
      prm->bucket_of[p] = b;
    }
  }
  __syncthreads();
  for (int i = threadIdx.x; i < kNumSubBuckets; i += blockDim.x)
    if (hist[i]) atomicAdd(&prm->scount[i], hist[i]);
}

// One block of kScanThreads, one thread per bucket and per queue position:
// bucket sizes and starts, the start of every (bucket, sub-bin) run inside
// its bucket, and the first work item of every queue position.
constexpr int kScanThreads = 256;
static_assert(kNumBuckets <= kScanThreads, "one thread per bucket");

// exclusive prefix sum over the block (Hillis-Steele in LDS); *total gets the sum
__device__ uint32_t block_exclusive_scan(uint32_t v, uint32_t* sh, uint32_t* total) {
  const int t = threadIdx.x;
  sh[t] = v;
  __syncthreads();
  for (int d = 1; d < kScanThreads; d <<= 1) {
    const uint32_t x = t >= d ? sh[t - d] : 0u;
    __syncthreads();
    sh[t] += x;
    __syncthreads();
  }
  const uint32_t incl = sh[t];
  *total = sh[kScanThreads - 1];
  __syncthreads();
  return incl - v;
}

__global__ __launch_bounds__(kScanThreads) void k_scan(const Params* __restrict__ prm) {
  __shared__ uint32_t cnt[kNumBuckets];
  __shared__ uint32_t sh[kScanThreads];
  const int b = threadIdx.x;
  uint32_t sub[kSubBins];
  uint32_t acc = 0;
  if (b < kNumBuckets) {
#pragma unroll
    for (int s = 0; s < kSubBins; ++s) {
      sub[s] = acc;
      acc += prm->scount[b * kSubBins + s];
    }
    cnt[b] = acc;
    prm->bcount[b] = acc;
  }
  uint32_t n_sorted;
  const uint32_t start = block_exclusive_scan(acc, sh, &n_sorted);  // also orders cnt[] before its reads
  // queue position q = b serves bucket qorder[q]
  uint32_t items = 0;
  if (b < kNumBuckets) {
    const int bq = (int)prm->qorder[b];
    const uint32_t ppi = (uint32_t)pairs_per_item(bucket_kind(bq), bucket_class(bq));
    items = (cnt[bq] + ppi - 1) / ppi;
  }
  uint32_t n_items;
  const uint32_t qs = block_exclusive_scan(items, sh, &n_items);
  if (b < kNumBuckets) {
    prm->qstart[b] = qs;
    prm->bstart[b] = start;
#pragma unroll
    for (int s = 0; s < kSubBins; ++s) prm->sfill[b * kSubBins + s] = start + sub[s];
  }
  if (b == 0) {
    prm->qstart[kNumBuckets] = n_items;
    prm->counters[kCtrItems] = n_items;
    for (int q = 0; q < kPersistParts; ++q) prm->counters[kCtrQueueHead + q] = 0;
    prm->counters[kCtrRerun] = 0;
  }
  (void)n_sorted;
}

// After the banded fills: the first work item of every queue position of
// the persistent buckets in the two side lists of the fills (fb: bands too
// wide for the refill; db: bands of 17-64 diagonals).
__global__ __launch_bounds__(kScanThreads) void k_sidescan(const Params* __restrict__ prm) {
  __shared__ uint32_t sh[kScanThreads];
  const int q = threadIdx.x;
#pragma unroll 1
  for (int list = 0; list < 2; ++list) {
    uint32_t* qstart = list ? prm->dbqstart : prm->fbqstart;
    uint32_t items = 0;
    if (q < kNumBuckets) {
      const int b = (int)prm->qorder[q];
      if (persistent_bucket(b)) {
        const int cls = list ? bucket_class(b) : fallback_class(bucket_class(b));
        const uint32_t ppi = (uint32_t)pairs_per_item(bucket_kind(b), cls);
        items = list ? (prm->dbwide[b] + ppi - 1) / ppi + (prm->dbcount[b] + ppi - 1) / ppi
                     : (prm->fbcount[b] + ppi - 1) / ppi;
      }
    }
    uint32_t total;
    const uint32_t qs = block_exclusive_scan(items, sh, &total);
    if (q < kNumBuckets) qstart[q] = qs;
    if (q == 0) qstart[kNumBuckets] = total;
    __syncthreads();
  }
}

__global__ __launch_bounds__(kPlanThreads) void k_scatter(const Params* __restrict__ prm) {
  __shared__ uint32_t cnt[kNumSubBuckets];
  __shared__ uint32_t base[kNumSubBuckets];
  for (int i = threadIdx.x; i < kNumSubBuckets; i += blockDim.x) cnt[i] = 0;
  __syncthreads();
  uint32_t b[kPlanPairsPerThread], rank[kPlanPairsPerThread];
#pragma unroll
  for (int rep = 0; rep < kPlanPairsPerThread; ++rep) {
    const int64_t p = ((int64_t)blockIdx.x * kPlanPairsPerThread + rep) * blockDim.x + threadIdx.x;
    b[rep] = kSkip;
    rank[rep] = 0;
    if (p < prm->n_pairs) {
      b[rep] = prm->bucket_of[p];
      if (b[rep] != kSkip) rank[rep] = atomicAdd(&cnt[b[rep]], 1u);
    }
  }
  __syncthreads();
  for (int i = threadIdx.x; i < kNumSubBuckets; i += blockDim.x)
    base[i] = cnt[i] ? atomicAdd(&prm->sfill[i], cnt[i]) : 0;
  __syncthreads();
#pragma unroll
  for (int rep = 0; rep < kPlanPairsPerThread; ++rep) {
    const int64_t p = ((int64_t)blockIdx.x * kPlanPairsPerThread + rep) * blockDim.x + threadIdx.x;
    if (b[rep] != kSkip) prm->sorted[base[b[rep]] + rank[rep]] = (uint32_t)p;
  }
}

__global__ __launch_bounds__(256) void k_pack2bit(const uint8_t* __restrict__ codes, int64_t n,
                                                   uint32_t* __restrict__ words) {
  const int64_t w = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const int64_t nw = (n + 15) / 16;
  if (w >= nw) return;
  uint32_t v = 0;
  const int64_t b0 = w * 16;
  for (int x = 0; x < 16; ++x) {
    const int64_t i = b0 + x;
    if (i < n) v |= ((uint32_t)codes[i] & 3u) << (2 * x);
  }
  words[w] = v;
}

}  // namespace mica

namespace mica {

// registration functions of the per-bucket fill kernels (one source file each)
#define MICA_FILL_DECL(kind, mode, dir) void reg_fill_##kind##_##mode##_##dir(KernelTable& t);
#define MICA_FILL_ALL(X) \
  X(k16, 0, 0) X(k16, 0, 1) X(k16, 1, 0) X(k16, 1, 1) \
  X(k16s, 0, 0) X(k16s, 0, 1) X(k16s, 1, 0) X(k16s, 1, 1) \
  X(k32, 0, 0) X(k32, 0, 1) X(k32, 1, 0) X(k32, 1, 1) \
  X(k16, 2, 0) X(k16, 2, 1) X(k16s, 2, 0) X(k16s, 2, 1) X(k32, 2, 0) X(k32, 2, 1)
MICA_FILL_ALL(MICA_FILL_DECL)
#define MICA_SIDE_ALL(X) X(k16, 0) X(k16, 1) X(k16, 2) X(k16s, 0) X(k16s, 1) X(k16s, 2) X(k32, 0) X(k32, 1) X(k32, 2)
#define MICA_SIDE_DECL(kind, mode) void reg_side_##kind##_##mode(KernelTable& t);
MICA_SIDE_ALL(MICA_SIDE_DECL)
#define MICA_PERSIST_ALL(X) \
  X(0, 0, 0) X(0, 0, 1) X(0, 1, 0) X(0, 1, 1) X(0, 2, 0) X(0, 2, 1) \
  X(1, 0, 0) X(1, 0, 1) X(1, 1, 0) X(1, 1, 1) X(1, 2, 0) X(1, 2, 1)
#define MICA_PERSIST_DECL(dir, mode, part) void reg_persistent_##dir##_##mode##_##part(KernelTable& t);
MICA_PERSIST_ALL(MICA_PERSIST_DECL)
#define MICA_PERSIST_SIDE_ALL(X) X(0, 0) X(0, 1) X(1, 0) X(1, 1) X(2, 0) X(2, 1)
#define MICA_PERSIST_SIDE_DECL(mode, part) void reg_persistent_side_##mode##_##part(KernelTable& t);
MICA_PERSIST_SIDE_ALL(MICA_PERSIST_SIDE_DECL)

KernelTable::KernelTable() {
#define MICA_FILL_CALL(kind, mode, dir) reg_fill_##kind##_##mode##_##dir(*this);
  MICA_FILL_ALL(MICA_FILL_CALL)
#define MICA_SIDE_CALL(kind, mode) reg_side_##kind##_##mode(*this);
  MICA_SIDE_ALL(MICA_SIDE_CALL)
#define MICA_PERSIST_CALL(dir, mode, part) reg_persistent_##dir##_##mode##_##part(*this);
  MICA_PERSIST_ALL(MICA_PERSIST_CALL)
#define MICA_PERSIST_SIDE_CALL(mode, part) reg_persistent_side_##mode##_##part(*this);
  MICA_PERSIST_SIDE_ALL(MICA_PERSIST_SIDE_CALL)
  sidescan = &k_sidescan;
  rerun[0] = &k_rerun<false>;
  rerun[1] = &k_rerun<true>;
  zero = &k_zero;
  plan = &k_plan;
  scan = &k_scan;
  scatter = &k_scatter;
}

const KernelTable& kernels() {
  static KernelTable t;
  return t;
}

hipError_t launch_pack2bit(const uint8_t* codes, int64_t n, uint32_t* words, hipStream_t s) {
  const int64_t nw = (n + 15) / 16;
  if (nw == 0) return hipSuccess;
  hipLaunchKernelGGL(k_pack2bit, dim3((unsigned)((nw + 255) / 256)), dim3(256), 0, s, codes, n, words);
  return hipGetLastError();
}

}  // namespace mica
