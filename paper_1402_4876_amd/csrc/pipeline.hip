// Host pipeline: FASTQ batches in, SAM records out, the few-mismatch search
// and the DP phase on the GPU in between.  One reader thread parses and packs
// batches, the calling thread enqueues each batch's GPU work on one of two
// slots (stream, DP context, buffers), and a writer thread waits for a
// batch, formats its records on several threads and writes them in order.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <atomic>
#include <charconv>
#include <chrono>
#include <condition_variable>
#include <cstdio>
#include <cstring>
#include <deque>
#include <memory>
#include <mutex>
#include <string>
#include <thread>
#include <vector>

#include <sys/mman.h>
#include <sys/stat.h>
#include <unistd.h>

#include "ctx.h"
#include "fm_common.h"
#include "mica_fm.h"
#include "mica_pipe.h"

namespace mica {
namespace {

constexpr int kCigCap = 32;           // CIGAR runs kept per DP window and per read
constexpr int64_t kMaxBatch = 4000000;

enum : int32_t { kUnmapped = 0, kBySearch = 1, kByDp = 2, kRepetitive = 3 };

// ---- kernels ----------------------------------------------------------------

// DP windows of the reads without a search hit: one per distinct seed
// placement (seeds within band of an earlier one of the same read are
// dropped), placement -/+ band clipped to the reference; unused slots get an
// empty read (a trivial pair the DP planner settles at once)
__global__ void k_make_pairs(int64_t n, const int32_t* __restrict__ len, const uint64_t* __restrict__ off,
                             const int32_t* __restrict__ best, const uint32_t* __restrict__ fst,
                             const int64_t* __restrict__ cand, int64_t L, int band, uint64_t* __restrict__ woff,
                             int32_t* __restrict__ wlen, uint64_t* __restrict__ roff2, int32_t* __restrict__ rlen2) {
  const int64_t r = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (r >= n) return;
  const int m = len[r];
  const bool need = fst[r] == 0 && best[r] < 0 && m > 0;
  int64_t c[3];
  for (int j = 0; j < 3; ++j) c[j] = cand[r * 3 + j];
  for (int j = 0; j < 3; ++j) {
    const int64_t s = r * 3 + j;
    bool ok = need && c[j] != MICA_FM_NO_CAND;
    for (int jj = 0; jj < j; ++jj) {
      if (ok && c[jj] != MICA_FM_NO_CAND) {
        const int64_t d = c[j] > c[jj] ? c[j] - c[jj] : c[jj] - c[j];
        if (d <= band) ok = false;
      }
    }
    int64_t ws = 0, we = 0;
    if (ok) {
      ws = c[j] - band;
      we = c[j] + m + band;
      ws = ws < 0 ? 0 : ws;
      we = we > L ? L : we;
      if (we <= ws) ok = false;
    }
    woff[s] = ok ? (uint64_t)ws : 0;
    wlen[s] = ok ? (int32_t)(we - ws) : 0;
    roff2[s] = off[r];
    rlen2[s] = ok ? m : 0;
  }
}

// per read: the search hit, else the best DP window (highest score, then the
// smallest reference start), its CIGAR compacted into cig_out
__global__ void k_pick(int64_t n, const int32_t* __restrict__ len, const int32_t* __restrict__ best,
                       const int32_t* __restrict__ nbest, const int64_t* __restrict__ pos,
                       const uint32_t* __restrict__ fst, const uint64_t* __restrict__ woff,
                       const int32_t* __restrict__ rlen2, const int32_t* __restrict__ score,
                       const int32_t* __restrict__ qstart, const uint32_t* __restrict__ dst,
                       const int32_t* __restrict__ ncig, const uint32_t* __restrict__ cig, int a, int b,
                       int min_score, int32_t* __restrict__ kind, int64_t* __restrict__ fpos,
                       int32_t* __restrict__ fscore, int32_t* __restrict__ fmm, int32_t* __restrict__ mapq,
                       int32_t* __restrict__ fncig, int32_t* __restrict__ cig_off, uint32_t* __restrict__ cig_out,
                       uint32_t* __restrict__ ctr) {
  const int64_t r = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (r >= n) return;
  const int m = len[r];
  int32_t k_ = kUnmapped, sc = 0, mm = 0, q = 0, nc = 0, co = 0;
  int64_t p = -1;
  if (fst[r] & MICA_ST_REPETITIVE) {
    k_ = kRepetitive;
  } else if (fst[r] == 0 && best[r] >= 0) {
    k_ = kBySearch;
    p = pos[r];
    mm = best[r];
    sc = (m - mm) * a + mm * b;
    q = nbest[r] == 1 ? 60 : 0;
  } else if (fst[r] == 0) {
    int bj = -1, cnt = 0;
    int32_t bs = 0;
    int64_t bp = 0;
    for (int j = 0; j < 3; ++j) {
      const int64_t s = r * 3 + j;
      if (rlen2[s] == 0 || (dst[s] & ~(uint32_t)MICA_ST_SATURATED) != 0) continue;
      const int64_t pj = (int64_t)woff[s] + qstart[s];
      if (bj < 0 || score[s] > bs) {
        bj = j;
        bs = score[s];
        bp = pj;
        cnt = 1;
      } else if (score[s] == bs) {
        ++cnt;
        if (pj < bp) {
          bj = j;
          bp = pj;
        }
      }
    }
    if (bj >= 0 && bs >= min_score) {
      const int64_t s = r * 3 + bj;
      k_ = kByDp;
      p = bp;
      sc = bs;
      q = cnt == 1 ? 60 : 0;
      nc = ncig[s];
      co = (int32_t)atomicAdd(ctr, (uint32_t)nc);
      for (int x = 0; x < nc; ++x) cig_out[co + x] = cig[s * kCigCap + x];
    }
  }
  kind[r] = k_;
  fpos[r] = p;
  fscore[r] = sc;
  fmm[r] = mm;
  mapq[r] = q;
  fncig[r] = nc;
  cig_off[r] = co;
}

// ---- host side --------------------------------------------------------------

struct HostBatch {
  int64_t n = 0;
  // names, sequences and qualities of the batch: offsets into the mapped
  // input file (mapped != nullptr), else into text, a copy of the lines
  const char* mapped = nullptr;
  std::string text;
  const char* base() const { return mapped ? mapped : text.data(); }
  std::vector<uint64_t> name_off, seq_off, qual_off;
  std::vector<int32_t> name_len, len;
  std::vector<uint8_t> non_acgt;
  std::vector<uint32_t> words;  // reads, 2-bit, each from a 16-base boundary
  std::vector<uint64_t> roff;
  std::vector<int32_t> dlen;    // read length sent to the device (0 for non-ACGT reads)
  int32_t max_m = 0;
};

template <class T>
struct Queue {
  std::mutex mu;
  std::condition_variable cv;
  std::deque<T> q;
  size_t cap = 2;
  void push(T v) {
    std::unique_lock<std::mutex> lk(mu);
    cv.wait(lk, [&] { return q.size() < cap; });
    q.push_back(std::move(v));
    cv.notify_all();
  }
  T pop() {
    std::unique_lock<std::mutex> lk(mu);
    cv.wait(lk, [&] { return !q.empty(); });
    T v = std::move(q.front());
    q.pop_front();
    cv.notify_all();
    return v;
  }
};

// FASTQ reader: whole lines of the file.  A regular file is mapped into
// memory and its lines are handed out in place (batches keep offsets into
// the mapping, which lives until the reader is destroyed: after every batch
// is written); anything else (a pipe) is read through a buffer, whose lines
// the batch copies.
struct LineReader {
  FILE* f = nullptr;
  std::vector<char> buf;
  size_t beg = 0, end = 0;
  bool eof = false;
  const char* map = nullptr;
  size_t map_len = 0;
  explicit LineReader(FILE* fp) : f(fp) {
    struct stat st;
    const int fd = fileno(fp);
    if (fd >= 0 && fstat(fd, &st) == 0 && S_ISREG(st.st_mode) && st.st_size > 0) {
      void* m = mmap(nullptr, (size_t)st.st_size, PROT_READ, MAP_PRIVATE, fd, 0);
      if (m != MAP_FAILED) {
        map = (const char*)m;
        map_len = (size_t)st.st_size;
        (void)madvise(m, map_len, MADV_SEQUENTIAL);
        return;
      }
    }
    buf.resize(size_t(16) << 20);
  }
  ~LineReader() {
    if (map) (void)munmap((void*)map, map_len);
  }
  LineReader(const LineReader&) = delete;
  LineReader& operator=(const LineReader&) = delete;
  // next line without its newline (nor a carriage return before it); false
  // at the end of the file
  bool next(const char** s, size_t* n) {
    if (map) {
      if (beg >= map_len) return false;
      const char* nl = (const char*)memchr(map + beg, '\n', map_len - beg);
      const size_t e = nl ? (size_t)(nl - map) : map_len;
      *s = map + beg;
      *n = e - beg;
      beg = nl ? e + 1 : map_len;
      if (*n && (*s)[*n - 1] == '\r') --*n;
      return true;
    }
    for (;;) {
      char* nl = (char*)memchr(buf.data() + beg, '\n', end - beg);
      if (nl) {
        *s = buf.data() + beg;
        *n = (size_t)(nl - (buf.data() + beg));
        beg = (size_t)(nl - buf.data()) + 1;
        if (*n && (*s)[*n - 1] == '\r') --*n;
        return true;
      }
      if (eof) {
        if (beg < end) {  // a last line without newline
          *s = buf.data() + beg;
          *n = end - beg;
          beg = end;
          return true;
        }
        return false;
      }
      if (beg > 0) {
        memmove(buf.data(), buf.data() + beg, end - beg);
        end -= beg;
        beg = 0;
      }
      if (end == buf.size()) buf.resize(buf.size() * 2);
      const size_t got = fread(buf.data() + end, 1, buf.size() - end, f);
      end += got;
      if (got == 0) eof = true;
    }
  }
};

// base code of a FASTQ letter (A0 C1 G2 T3, either case), -1 for any other
struct CodeTable {
  int8_t v[256];
  CodeTable() {
    for (int i = 0; i < 256; ++i) v[i] = -1;
    v['A'] = v['a'] = 0;
    v['C'] = v['c'] = 1;
    v['G'] = v['g'] = 2;
    v['T'] = v['t'] = 3;
  }
};
const CodeTable kCodes;
inline int code_of(char c) { return kCodes.v[(uint8_t)c]; }

struct Slot {
  hipStream_t stream = nullptr;
  mica_ctx_t ctx = nullptr;
  hipEvent_t ev_start = nullptr, ev_done = nullptr;
  // capacity of the read-word buffers
  size_t word_cap = 0;
  uint32_t *d_words = nullptr, *h_words = nullptr;
  uint64_t *d_off = nullptr, *h_off = nullptr;
  int32_t *d_len = nullptr, *h_len = nullptr;
  // search outputs
  int32_t *d_best = nullptr, *d_nbest = nullptr, *d_nhits = nullptr;
  int64_t *d_pos = nullptr, *d_cand = nullptr;
  uint32_t* d_fst = nullptr;
  // DP pairs and outputs (3 per read)
  uint64_t *d_woff = nullptr, *d_roff2 = nullptr;
  int32_t *d_wlen = nullptr, *d_rlen2 = nullptr;
  int32_t *d_score = nullptr, *d_rs = nullptr, *d_re = nullptr, *d_qs = nullptr, *d_qe = nullptr, *d_ncig = nullptr;
  uint32_t *d_dst = nullptr, *d_cig = nullptr;
  // per-read results, device and pinned host (one block: 7 arrays + counter)
  void* d_res = nullptr;
  void* h_res = nullptr;
  uint32_t *d_cig_out = nullptr, *h_cig = nullptr;
  // slot free for the next batch
  std::mutex mu;
  std::condition_variable cv;
  bool busy = false;
};

// byte offsets of the per-read result arrays in a result block of n reads
struct ResLayout {
  size_t kind, pos, score, mm, mapq, ncig, cig_off, ctr, total;
  explicit ResLayout(int64_t n) {
    size_t o = 0;
    auto take = [&](size_t bytes) {
      const size_t at = o;
      o = align_up(o + bytes, 256);
      return at;
    };
    kind = take(4 * n);
    pos = take(8 * n);
    score = take(4 * n);
    mm = take(4 * n);
    mapq = take(4 * n);
    ncig = take(4 * n);
    cig_off = take(4 * n);
    ctr = take(4);
    total = o;
  }
};

}  // namespace
}  // namespace mica

struct mica_pipe {
  int device = 0;
  mica_pipe_params_t prm{};
  std::string ref_name;
  uint64_t ref_len = 0;
  std::vector<uint32_t> ref_words;  // host copy for the NM of DP alignments
  mica_fm_t fm = nullptr;
  mica::Slot slot[2];
};

namespace mica {
namespace {

#define PIPE_HIP(expr)                                                                           \
  do {                                                                                          \
    hipError_t e_ = (expr);                                                                     \
    if (e_ != hipSuccess) return fail(MICA_ERR_HIP, std::string(#expr) + ": " + hipGetErrorString(e_)); \
  } while (0)

template <class T>
mica_status_t dalloc(T** p, size_t count) {
  PIPE_HIP(hipMalloc((void**)p, std::max<size_t>(count, 1) * sizeof(T)));
  return MICA_OK;
}

mica_status_t slot_alloc(Slot& s, int device, int64_t nmax) {
  PIPE_HIP(hipSetDevice(device));
  PIPE_HIP(hipStreamCreateWithFlags(&s.stream, hipStreamNonBlocking));
  PIPE_HIP(hipEventCreate(&s.ev_start));
  PIPE_HIP(hipEventCreate(&s.ev_done));
  mica_status_t st = mica_ctx_create(device, 0, &s.ctx);
  if (st != MICA_OK) return st;
  const size_t n = (size_t)nmax, n3 = 3 * n;
#define PA(ptr, cnt)                          \
  do {                                        \
    mica_status_t e2 = dalloc(&(ptr), (cnt)); \
    if (e2 != MICA_OK) return e2;             \
  } while (0)
  PA(s.d_off, n); PA(s.d_len, n);
  PA(s.d_best, n); PA(s.d_nbest, n); PA(s.d_nhits, n); PA(s.d_pos, n); PA(s.d_fst, n); PA(s.d_cand, n3);
  PA(s.d_woff, n3); PA(s.d_roff2, n3); PA(s.d_wlen, n3); PA(s.d_rlen2, n3);
  PA(s.d_score, n3); PA(s.d_rs, n3); PA(s.d_re, n3); PA(s.d_qs, n3); PA(s.d_qe, n3); PA(s.d_ncig, n3);
  PA(s.d_dst, n3); PA(s.d_cig, n3 * kCigCap);
  PA(s.d_cig_out, n * kCigCap);
#undef PA
  const ResLayout lay(nmax);
  PIPE_HIP(hipMalloc(&s.d_res, lay.total));
  PIPE_HIP(hipHostMalloc(&s.h_res, lay.total, hipHostMallocDefault));
  PIPE_HIP(hipHostMalloc((void**)&s.h_cig, n * kCigCap * 4, hipHostMallocDefault));
  PIPE_HIP(hipHostMalloc((void**)&s.h_off, n * 8, hipHostMallocDefault));
  PIPE_HIP(hipHostMalloc((void**)&s.h_len, n * 4, hipHostMallocDefault));
  return MICA_OK;
}

void slot_free(Slot& s) {
  if (s.stream) (void)hipStreamSynchronize(s.stream);
  void* dev[] = {s.d_words, s.d_off, s.d_len, s.d_best, s.d_nbest, s.d_nhits, s.d_pos, s.d_cand, s.d_fst,
                 s.d_woff, s.d_roff2, s.d_wlen, s.d_rlen2, s.d_score, s.d_rs, s.d_re, s.d_qs, s.d_qe,
                 s.d_ncig, s.d_dst, s.d_cig, s.d_res, s.d_cig_out};
  for (void* p : dev)
    if (p) (void)hipFree(p);
  void* host[] = {s.h_words, s.h_off, s.h_len, s.h_res, s.h_cig};
  for (void* p : host)
    if (p) (void)hipHostFree(p);
  if (s.ctx) mica_ctx_destroy(s.ctx);
  if (s.ev_start) (void)hipEventDestroy(s.ev_start);
  if (s.ev_done) (void)hipEventDestroy(s.ev_done);
  if (s.stream) (void)hipStreamDestroy(s.stream);
}

mica_status_t ensure_words(Slot& s, size_t words) {
  if (words <= s.word_cap) return MICA_OK;
  const size_t cap = std::max(words, s.word_cap * 2);
  if (s.d_words) PIPE_HIP(hipFree(s.d_words));
  if (s.h_words) PIPE_HIP(hipHostFree(s.h_words));
  s.d_words = nullptr;
  s.h_words = nullptr;
  PIPE_HIP(hipMalloc((void**)&s.d_words, cap * 4));
  PIPE_HIP(hipHostMalloc((void**)&s.h_words, cap * 4, hipHostMallocDefault));
  s.word_cap = cap;
  return MICA_OK;
}

// parse up to max_reads FASTQ records (record lines on this thread, the 2-bit
// packing on `threads` threads); *bad set for malformed input
std::unique_ptr<HostBatch> parse_batch(LineReader& in, int64_t max_reads, int threads, bool* bad) {
  auto b = std::make_unique<HostBatch>();
  b->mapped = in.map;
  b->name_off.reserve((size_t)max_reads);
  b->seq_off.reserve((size_t)max_reads);
  b->qual_off.reserve((size_t)max_reads);
  b->name_len.reserve((size_t)max_reads);
  b->len.reserve((size_t)max_reads);
  // offset of a line: in place in the mapping, else appended to the copy
  auto keep = [&](const char* p, size_t len) -> uint64_t {
    if (in.map) return (uint64_t)(p - in.map);
    const uint64_t o = b->text.size();
    b->text.append(p, len);
    return o;
  };
  const char* s;
  size_t n;
  while (b->n < max_reads) {
    if (!in.next(&s, &n)) break;
    if (n == 0) continue;  // blank line between records
    if (s[0] != '@') {
      *bad = true;
      return b;
    }
    size_t nl = 1;
    while (nl < n && s[nl] != ' ' && s[nl] != '\t') ++nl;
    b->name_off.push_back(keep(s + 1, nl - 1));
    b->name_len.push_back((int32_t)(nl - 1));
    const char* q;
    size_t qn;
    if (!in.next(&q, &qn)) {
      *bad = true;
      return b;
    }
    b->seq_off.push_back(keep(q, qn));
    b->len.push_back((int32_t)qn);
    if (!in.next(&q, &qn) || qn == 0 || q[0] != '+') {
      *bad = true;
      return b;
    }
    if (!in.next(&q, &qn) || (int64_t)qn != (int64_t)b->len.back()) {
      *bad = true;
      return b;
    }
    b->qual_off.push_back(keep(q, qn));
    b->n++;
  }
  // 2-bit packing, each read from a 16-base boundary
  b->roff.resize(b->n);
  b->dlen.resize(b->n);
  b->non_acgt.assign(b->n, 0);
  uint64_t tot = 0;
  for (int64_t r = 0; r < b->n; ++r) {
    b->roff[r] = tot;
    tot += ((uint64_t)b->len[r] + 15) / 16 * 16;
  }
  b->words.assign(std::max<uint64_t>(tot / 16, 1), 0u);
  std::vector<int32_t> part_max((size_t)threads, 0);
  auto pack = [&](int th, int64_t lo, int64_t hi) {
    int32_t mx = 0;
    for (int64_t r = lo; r < hi; ++r) {
      const char* sq = b->base() + b->seq_off[r];
      const int m = b->len[r];
      uint32_t* w = b->words.data() + b->roff[r] / 16;
      bool ok = true;
      for (int t0 = 0; t0 < m && ok; t0 += 16) {
        uint32_t word = 0;
        const int e = std::min(m - t0, 16);
        for (int t = 0; t < e; ++t) {
          const int c = code_of(sq[t0 + t]);
          ok = ok && c >= 0;
          word |= (uint32_t)(c & 3) << (2 * t);
        }
        w[t0 >> 4] = word;
      }
      b->non_acgt[r] = ok ? 0 : 1;
      b->dlen[r] = ok ? m : 0;
      if (ok) mx = std::max(mx, m);
    }
    part_max[(size_t)th] = mx;
  };
  const int T = (int)std::max<int64_t>(1, std::min<int64_t>(threads, b->n / 4096 + 1));
  const int64_t chunk = (b->n + T - 1) / T;
  std::vector<std::thread> th;
  for (int t = 1; t < T; ++t)
    th.emplace_back(pack, t, std::min<int64_t>(b->n, t * chunk), std::min<int64_t>(b->n, (t + 1) * chunk));
  pack(0, 0, std::min<int64_t>(b->n, chunk));
  for (auto& x : th) x.join();
  for (int32_t v : part_max) b->max_m = std::max(b->max_m, v);
  return b;
}

mica_status_t enqueue_batch(mica_pipe* P, Slot& s, const HostBatch& b) {
  const mica_pipe_params_t& pr = P->prm;
  const int64_t n = b.n;
  PIPE_HIP(hipSetDevice(P->device));
  mica_status_t st = ensure_words(s, b.words.size());
  if (st != MICA_OK) return st;
  std::memcpy(s.h_words, b.words.data(), b.words.size() * 4);
  std::memcpy(s.h_off, b.roff.data(), (size_t)n * 8);
  std::memcpy(s.h_len, b.dlen.data(), (size_t)n * 4);
  PIPE_HIP(hipEventRecord(s.ev_start, s.stream));
  PIPE_HIP(hipMemcpyAsync(s.d_words, s.h_words, b.words.size() * 4, hipMemcpyHostToDevice, s.stream));
  PIPE_HIP(hipMemcpyAsync(s.d_off, s.h_off, (size_t)n * 8, hipMemcpyHostToDevice, s.stream));
  PIPE_HIP(hipMemcpyAsync(s.d_len, s.h_len, (size_t)n * 4, hipMemcpyHostToDevice, s.stream));
  // 1. few-mismatch search
  mica_fm_batch_t fb;
  std::memset(&fb, 0, sizeof(fb));
  fb.reads2b = s.d_words;
  fb.reads_len = (uint64_t)b.words.size() * 16;
  fb.read_off = s.d_off;
  fb.read_len = s.d_len;
  fb.n_reads = n;
  fb.k = pr.k;
  fb.max_occ = pr.max_occ;
  fb.best_mm = s.d_best;
  fb.n_best = s.d_nbest;
  fb.n_hits = s.d_nhits;
  fb.pos = s.d_pos;
  fb.status = s.d_fst;
  fb.cand = s.d_cand;
  st = mica_fm_search(P->fm, &fb, s.stream);
  if (st != MICA_OK) return st;
  // 2. DP windows of the reads without a hit
  const unsigned blocks = (unsigned)((n + 255) / 256);
  hipLaunchKernelGGL(k_make_pairs, dim3(blocks), dim3(256), 0, s.stream, n, s.d_len, s.d_off, s.d_best, s.d_fst,
                     s.d_cand, (int64_t)P->ref_len, pr.band, s.d_woff, s.d_wlen, s.d_roff2, s.d_rlen2);
  PIPE_HIP(hipGetLastError());
  mica_batch_t db;
  std::memset(&db, 0, sizeof(db));
  db.ref2b = fm_index_of(P->fm)->ref2b;
  db.ref_len = P->ref_len;
  db.win_off = s.d_woff;
  db.win_len = s.d_wlen;
  db.reads2b = s.d_words;
  db.reads_len = fb.reads_len;
  db.read_off = s.d_roff2;
  db.read_len = s.d_rlen2;
  db.default_mode = MICA_MODE_SEMIGLOBAL;
  db.n_pairs = 3 * n;
  db.max_read_len = std::max(1, std::min(b.max_m, (int32_t)MICA_MAX_READ_LEN));
  db.max_win_len = std::min<int32_t>(MICA_MAX_WIN_LEN, db.max_read_len + 2 * pr.band);
  db.score = s.d_score;
  db.read_end = s.d_re;
  db.ref_end = s.d_qe;
  db.read_start = s.d_rs;
  db.ref_start = s.d_qs;
  db.cigar = s.d_cig;
  db.cigar_cap = kCigCap;
  db.n_cigar = s.d_ncig;
  db.status = s.d_dst;
  st = mica_dp_align_batch(s.ctx, &db, &pr.scoring, MICA_OUT_CIGAR, s.stream);
  if (st != MICA_OK) return st;
  // 3. per-read choice, compacted CIGARs
  const ResLayout lay(n);
  char* R = (char*)s.d_res;
  PIPE_HIP(hipMemsetAsync(R + lay.ctr, 0, 4, s.stream));
  hipLaunchKernelGGL(k_pick, dim3(blocks), dim3(256), 0, s.stream, n, s.d_len, s.d_best, s.d_nbest, s.d_pos,
                     s.d_fst, s.d_woff, s.d_rlen2, s.d_score, s.d_qs, s.d_dst, s.d_ncig, s.d_cig,
                     pr.scoring.match, pr.scoring.mismatch, pr.min_score, (int32_t*)(R + lay.kind),
                     (int64_t*)(R + lay.pos), (int32_t*)(R + lay.score), (int32_t*)(R + lay.mm),
                     (int32_t*)(R + lay.mapq), (int32_t*)(R + lay.ncig), (int32_t*)(R + lay.cig_off), s.d_cig_out,
                     (uint32_t*)(R + lay.ctr));
  PIPE_HIP(hipGetLastError());
  PIPE_HIP(hipMemcpyAsync(s.h_res, s.d_res, lay.total, hipMemcpyDeviceToHost, s.stream));
  PIPE_HIP(hipEventRecord(s.ev_done, s.stream));
  return MICA_OK;
}

inline uint32_t ref_base(const mica_pipe* P, uint64_t p) { return (P->ref_words[p >> 4] >> (2 * (p & 15))) & 3u; }

// SAM records of reads [lo, hi) of a finished batch
// decimal text of v appended to out
inline void append_int(std::string* out, long long v) {
  char buf[24];
  const auto r = std::to_chars(buf, buf + sizeof(buf), v);
  out->append(buf, (size_t)(r.ptr - buf));
}

void format_range(const mica_pipe* P, const HostBatch& b, const char* res, const uint32_t* cig, int64_t lo,
                  int64_t hi, std::string* out) {
  const ResLayout lay(b.n);
  const int32_t* kind = (const int32_t*)(res + lay.kind);
  const int64_t* pos = (const int64_t*)(res + lay.pos);
  const int32_t* score = (const int32_t*)(res + lay.score);
  const int32_t* mm = (const int32_t*)(res + lay.mm);
  const int32_t* mapq = (const int32_t*)(res + lay.mapq);
  const int32_t* ncig = (const int32_t*)(res + lay.ncig);
  const int32_t* coff = (const int32_t*)(res + lay.cig_off);
  for (int64_t r = lo; r < hi; ++r) {
    const char* T = b.base();
    out->append(T + b.name_off[r], (size_t)b.name_len[r]);
    const int m = b.len[r];
    const int k_ = b.non_acgt[r] ? kUnmapped : kind[r];
    if (k_ == kBySearch || k_ == kByDp) {
      out->append("\t0\t");
      out->append(P->ref_name);
      out->push_back('\t');
      append_int(out, (long long)pos[r] + 1);
      out->push_back('\t');
      append_int(out, mapq[r]);
      out->push_back('\t');
      int nm = 0;
      if (k_ == kBySearch) {
        append_int(out, m);
        out->push_back('M');
        nm = mm[r];
      } else {
        // NM: mismatches in M runs plus inserted and deleted bases
        uint64_t rp = (uint64_t)pos[r];
        int qp = 0;
        const char* sq = T + b.seq_off[r];
        for (int x = 0; x < ncig[r]; ++x) {
          const uint32_t w = cig[coff[r] + x];
          const int L = (int)(w >> 4), op = (int)(w & 15);
          append_int(out, L);
          out->push_back(op == 0 ? 'M' : (op == 1 ? 'I' : 'D'));
          if (op == 0) {
            for (int t = 0; t < L; ++t) nm += (uint32_t)code_of(sq[qp + t]) != ref_base(P, rp + t);
            qp += L;
            rp += L;
          } else if (op == 1) {
            nm += L;
            qp += L;
          } else {
            nm += L;
            rp += L;
          }
        }
      }
      out->append("\t*\t0\t0\t");
      out->append(T + b.seq_off[r], (size_t)m);
      out->push_back('\t');
      out->append(T + b.qual_off[r], (size_t)m);
      out->append("\tNM:i:");
      append_int(out, nm);
      out->append("\tAS:i:");
      append_int(out, score[r]);
      out->push_back('\n');
    } else {
      out->append("\t4\t*\t0\t0\t*\t*\t0\t0\t");
      if (m == 0) {
        out->append("*\t*\n");
      } else {
        out->append(T + b.seq_off[r], (size_t)m);
        out->push_back('\t');
        out->append(T + b.qual_off[r], (size_t)m);
        out->push_back('\n');
      }
    }
  }
}

double since(std::chrono::steady_clock::time_point t0) {
  return std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
}

}  // namespace
}  // namespace mica

extern "C" mica_status_t mica_pipe_create(int hip_device, const uint32_t* host_ref2b, uint64_t ref_len,
                                          const char* ref_name, const mica_pipe_params_t* prm, mica_pipe_t* out) {
  using namespace mica;
  if (!out || !prm || !host_ref2b || !ref_name) return fail(MICA_ERR_INVALID_ARG, "NULL argument");
  *out = nullptr;
  if (prm->k < 0 || prm->k > 2 || prm->max_occ < 1 || prm->max_occ > MICA_FM_MAX_OCC || prm->band < 0 ||
      prm->band > 3000 || prm->batch_reads < 1 || prm->batch_reads > kMaxBatch || prm->format_threads < 1 ||
      prm->format_threads > 64)
    return fail(MICA_ERR_INVALID_ARG, "pipeline parameter out of range");
  if (!*ref_name || strpbrk(ref_name, " \t\n")) return fail(MICA_ERR_INVALID_ARG, "reference name empty or with blanks");
  auto P = std::make_unique<mica_pipe>();
  P->device = hip_device;
  P->prm = *prm;
  P->ref_name = ref_name;
  P->ref_len = ref_len;
  P->ref_words.assign(host_ref2b, host_ref2b + (ref_len + 15) / 16);
  mica_status_t st = mica_fm_create(hip_device, host_ref2b, ref_len, &P->fm);
  if (st != MICA_OK) return st;
  for (auto& s : P->slot) {
    st = slot_alloc(s, hip_device, prm->batch_reads);
    if (st != MICA_OK) {
      for (auto& t : P->slot) slot_free(t);
      mica_fm_destroy(P->fm);
      return st;
    }
  }
  *out = P.release();
  return MICA_OK;
}

extern "C" mica_status_t mica_pipe_destroy(mica_pipe_t P) {
  if (!P) return MICA_OK;
  (void)hipSetDevice(P->device);
  for (auto& s : P->slot) mica::slot_free(s);
  mica_fm_destroy(P->fm);
  delete P;
  return MICA_OK;
}

extern "C" mica_status_t mica_pipe_run(mica_pipe_t P, const char* fastq_path, const char* sam_path,
                                       mica_pipe_stats_t* stats) {
  using namespace mica;
  if (!P || !fastq_path || !sam_path) return fail(MICA_ERR_INVALID_ARG, "NULL argument");
  const auto t0 = std::chrono::steady_clock::now();
  FILE* fin = fopen(fastq_path, "rb");
  if (!fin) return fail(MICA_ERR_INVALID_ARG, std::string("cannot open ") + fastq_path);
  FILE* fout = fopen(sam_path, "wb");
  if (!fout) {
    fclose(fin);
    return fail(MICA_ERR_INVALID_ARG, std::string("cannot create ") + sam_path);
  }
  {
    std::string h = "@HD\tVN:1.6\tSO:unsorted\n@SQ\tSN:" + P->ref_name + "\tLN:" + std::to_string(P->ref_len) +
                    "\n@PG\tID:mica-mi355x\tPN:mica-mi355x\n";
    fwrite(h.data(), 1, h.size(), fout);
  }
  // A seekable SAM file takes each batch's formatted parts with one pwrite
  // per format thread at their offsets (the copies into the page cache run
  // in parallel); anything else (a pipe) takes them in order through fout.
  int64_t wpos = -1;
  if (fflush(fout) == 0) wpos = (int64_t)ftello(fout);
  const bool positional = wpos >= 0 && lseek(fileno(fout), 0, SEEK_CUR) >= 0;
  mica_pipe_stats_t S;
  std::memset(&S, 0, sizeof(S));
  std::atomic<int> err_status{MICA_OK};
  std::string err_msg;
  std::mutex err_mu;
  auto set_err = [&](mica_status_t st, const std::string& msg) {
    std::lock_guard<std::mutex> lk(err_mu);
    if (err_status.load() == MICA_OK) {
      err_status.store(st);
      err_msg = msg;
    }
  };
  using BatchPtr = std::unique_ptr<HostBatch>;
  Queue<BatchPtr> parsed;
  struct Done {
    BatchPtr b;
    int slot;
  };
  Queue<Done> gpu_done;
  gpu_done.cap = 2;

  // reader (the mapping of the input lives until this function returns,
  // after the writer has formatted every batch)
  LineReader in(fin);
  double parse_s = 0;
  std::thread reader([&] {
    for (;;) {
      const auto tp = std::chrono::steady_clock::now();
      bool bad = false;
      BatchPtr b = parse_batch(in, P->prm.batch_reads, P->prm.format_threads, &bad);
      parse_s += since(tp);
      if (bad) {
        set_err(MICA_ERR_INVALID_ARG, "malformed FASTQ record");
        b->n = 0;
      }
      const bool last = b->n == 0 || err_status.load() != MICA_OK;
      if (last) {
        parsed.push(nullptr);
        return;
      }
      parsed.push(std::move(b));
    }
  });

  // writer
  double fmt_s = 0, gpu_s = 0;
  std::thread writer([&] {
    // formatted SAM text per format thread, kept across batches so that
    // their memory is reused instead of faulted in again for every batch
    std::vector<std::string> parts((size_t)P->prm.format_threads);
    for (;;) {
      Done d = gpu_done.pop();
      if (!d.b) return;
      Slot& s = P->slot[d.slot];
      const HostBatch& b = *d.b;
      if (hipEventSynchronize(s.ev_done) != hipSuccess) set_err(MICA_ERR_HIP, "batch failed on the device");
      float ms = 0;
      if (hipEventElapsedTime(&ms, s.ev_start, s.ev_done) == hipSuccess) gpu_s += ms * 1e-3;
      const auto tf = std::chrono::steady_clock::now();
      if (err_status.load() == MICA_OK) {
        const ResLayout lay(b.n);
        const uint32_t used = *(const uint32_t*)((const char*)s.h_res + lay.ctr);
        if (used > (uint64_t)b.n * kCigCap ||
            (used && hipMemcpy(s.h_cig, s.d_cig_out, (size_t)used * 4, hipMemcpyDeviceToHost) != hipSuccess)) {
          set_err(MICA_ERR_HIP, "CIGAR copy failed");
        } else {
          const int T = P->prm.format_threads;
          for (auto& x : parts) x.clear();
          std::vector<std::thread> th;
          const int64_t chunk = (b.n + T - 1) / T;
          for (int t = 0; t < T; ++t) {
            const int64_t lo = std::min<int64_t>(b.n, t * chunk), hi = std::min<int64_t>(b.n, lo + chunk);
            th.emplace_back([&, t, lo, hi] {
              parts[(size_t)t].reserve((size_t)(hi - lo) * 400);
              format_range(P, b, (const char*)s.h_res, s.h_cig, lo, hi, &parts[(size_t)t]);
            });
          }
          for (auto& x : th) x.join();
          if (positional) {
            std::vector<int64_t> at((size_t)T);
            for (int t = 0; t < T; ++t) {
              at[(size_t)t] = wpos;
              wpos += (int64_t)parts[(size_t)t].size();
            }
            std::atomic<bool> ok{true};
            th.clear();
            for (int t = 0; t < T; ++t)
              th.emplace_back([&, t] {
                const std::string& x = parts[(size_t)t];
                size_t done = 0;
                while (done < x.size()) {
                  const ssize_t w = pwrite(fileno(fout), x.data() + done, x.size() - done, (off_t)(at[(size_t)t] + (int64_t)done));
                  if (w <= 0) {
                    ok = false;
                    return;
                  }
                  done += (size_t)w;
                }
              });
            for (auto& x : th) x.join();
            if (!ok) set_err(MICA_ERR_INVALID_ARG, "SAM write failed");
          } else {
            for (auto& x : parts)
              if (fwrite(x.data(), 1, x.size(), fout) != x.size()) set_err(MICA_ERR_INVALID_ARG, "SAM write failed");
          }
          const int32_t* kind = (const int32_t*)((const char*)s.h_res + lay.kind);
          for (int64_t r = 0; r < b.n; ++r) {
            const int k_ = b.non_acgt[r] ? kUnmapped : kind[r];
            S.mapped_search += k_ == kBySearch;
            S.mapped_dp += k_ == kByDp;
            S.unmapped += k_ != kBySearch && k_ != kByDp;
            S.non_acgt += b.non_acgt[r];
            S.repetitive += k_ == kRepetitive;
          }
          S.reads += b.n;
          S.batches++;
        }
      }
      fmt_s += since(tf);
      {
        std::lock_guard<std::mutex> lk(s.mu);
        s.busy = false;
      }
      s.cv.notify_all();
    }
  });

  // GPU driver: batches alternate between the two slots
  int64_t i = 0;
  for (;;) {
    BatchPtr b = parsed.pop();
    if (!b) break;
    Slot& s = P->slot[i & 1];
    {
      std::unique_lock<std::mutex> lk(s.mu);
      s.cv.wait(lk, [&] { return !s.busy; });
      s.busy = true;
    }
    if (err_status.load() == MICA_OK) {
      if (b->n > P->prm.batch_reads) {
        set_err(MICA_ERR_LIMIT, "batch larger than the slots");
      } else {
        const mica_status_t st = enqueue_batch(P, s, *b);
        if (st != MICA_OK) set_err(st, mica_last_error());
      }
    }
    if (err_status.load() != MICA_OK) {
      std::lock_guard<std::mutex> lk(s.mu);
      s.busy = false;
      // drain the reader so it can finish
      continue;
    }
    gpu_done.push(Done{std::move(b), (int)(i & 1)});
    ++i;
  }
  gpu_done.push(Done{nullptr, 0});
  reader.join();
  writer.join();
  fclose(fin);
  if (fclose(fout) != 0) set_err(MICA_ERR_INVALID_ARG, "SAM close failed");
  S.seconds = since(t0);
  S.parse_seconds = parse_s;
  S.gpu_seconds = gpu_s;
  S.format_seconds = fmt_s;
  if (stats) *stats = S;
  if (err_status.load() != MICA_OK) return fail((mica_status_t)err_status.load(), err_msg);
  return MICA_OK;
}
