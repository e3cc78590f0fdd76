// Autotuner of a context's kernel plan (read length -> lanes per pair and rows
// per lane) and the plan file.
//
// The plan decides only how the DP of a pair is laid out on the GPU (see the
// kernel classes), never its result, so the tuner keeps a candidate only if
// its outputs equal those of the default plan on every pair of the sample,
// and among those it takes the fastest.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cctype>
#include <cstdio>
#include <cstring>
#include <string>
#include <vector>

#include "ctx.h"
#include "dp_common.h"
#include "mica_dp.h"

using namespace mica;

namespace {

constexpr int kRangeWidth = 16;       // read lengths per tuned range
constexpr int kMinPairs = 256;        // ranges with fewer sample pairs keep their plan
constexpr int kMaxTunePairs = 65536;  // sample pairs per range in the tuning batch
constexpr double kMinGain = 0.01;     // a new plan must be this much faster

// device buffers of one sub-batch and its outputs
struct TuneBuffers {
  uint64_t* win_off = nullptr;
  int32_t* win_len = nullptr;
  uint64_t* read_off = nullptr;
  int32_t* read_len = nullptr;
  uint8_t* mode = nullptr;
  int32_t* ext_h0 = nullptr;
  int32_t* out = nullptr;  // 7 arrays of n: score, read_end, ref_end, read_start, ref_start, n_cigar, status
  uint32_t* cigar = nullptr;
  ~TuneBuffers() {
    for (void* p : {(void*)win_off, (void*)win_len, (void*)read_off, (void*)read_len, (void*)mode,
                    (void*)ext_h0, (void*)out, (void*)cigar})
      if (p) (void)hipFree(p);
  }
};

struct HostOutputs {
  std::vector<int32_t> v;      // 7 * n
  std::vector<uint32_t> cigar;  // n * cap
};

bool same_outputs(const HostOutputs& a, const HostOutputs& b, int64_t n, int cap, bool cigar) {
  if (a.v != b.v) return false;
  if (!cigar) return true;
  const int32_t* ncig = a.v.data() + 5 * n;
  for (int64_t p = 0; p < n; ++p) {
    const int64_t k = std::min<int64_t>(ncig[p] < 0 ? -(int64_t)ncig[p] : ncig[p], cap);
    for (int64_t x = 0; x < k; ++x)
      if (a.cigar[p * cap + x] != b.cigar[p * cap + x]) return false;
  }
  return true;
}

template <class T>
mica_status_t to_host(std::vector<T>* dst, const T* src, int64_t n) {
  dst->resize((size_t)n);
  if (n) HIP_TRY(hipMemcpy(dst->data(), src, (size_t)n * sizeof(T), hipMemcpyDeviceToHost));
  return MICA_OK;
}

template <class T>
mica_status_t gather_up(T* dst, const std::vector<T>& src, const std::vector<int64_t>& idx) {
  std::vector<T> tmp(idx.size());
  for (size_t i = 0; i < idx.size(); ++i) tmp[i] = src[(size_t)idx[i]];
  HIP_TRY(hipMemcpy(dst, tmp.data(), tmp.size() * sizeof(T), hipMemcpyHostToDevice));
  return MICA_OK;
}

// the device copy of the plan table; batches still queued finish first (their
// fill kernels were chosen from the table they were enqueued with)
mica_status_t upload_plan(mica_ctx* c) {
  HIP_TRY(hipSetDevice(c->device));
  HIP_TRY(hipDeviceSynchronize());
  HIP_TRY(hipMemcpy(c->d_class, c->class_of_m, kMaxM + 1, hipMemcpyHostToDevice));
  return MICA_OK;
}

// candidate classes of the range [m_lo, m_hi], default first
std::vector<int> candidates(int m_hi) {
  std::vector<int> out;
  out.push_back(default_class_of(m_hi));
  const int r0 = (m_hi + 15) / 16;
  for (int r = r0; r <= std::min(r0 + 1, 16); ++r) out.push_back(class_of(16, r));
  for (int r : {4, 8, 16})
    if (64 * r >= m_hi) out.push_back(class_of(64, r));
  std::vector<int> uniq;
  for (int x : out)
    if (x >= 0 && std::find(uniq.begin(), uniq.end(), x) == uniq.end()) uniq.push_back(x);
  return uniq;
}

}  // namespace

extern "C" {

mica_status_t mica_ctx_autotune(mica_ctx_t c, const mica_batch_t* sample, const mica_scoring_t* scoring,
                                uint32_t flags, void* stream_, int32_t reps, mica_tune_entry_t* out,
                                int32_t out_cap, int32_t* n_out) {
  if (!c || !sample || !scoring || !n_out) return fail(MICA_ERR_INVALID_ARG, "NULL ctx, sample, scoring or n_out");
  if (reps < 1 || out_cap < 0) return fail(MICA_ERR_INVALID_ARG, "reps must be >= 1 and out_cap >= 0");
  *n_out = 0;
  const int64_t n = sample->n_pairs;
  if (n < 0) return fail(MICA_ERR_INVALID_ARG, "n_pairs < 0");
  if (n == 0) return MICA_OK;
  if (!sample->win_off || !sample->win_len || !sample->read_off || !sample->read_len)
    return fail(MICA_ERR_INVALID_ARG, "NULL sample descriptor array");
  if (sample->max_read_len < 1 || sample->max_read_len > kMaxM || sample->max_win_len < 0 ||
      sample->max_win_len > kMaxN)
    return fail(MICA_ERR_LIMIT, "max_read_len / max_win_len beyond the library limits");
  hipStream_t stream = (hipStream_t)stream_;
  HIP_TRY(hipSetDevice(c->device));
  HIP_TRY(hipStreamSynchronize(stream));

  std::vector<uint64_t> h_woff, h_roff;
  std::vector<int32_t> h_wlen, h_rlen;
  std::vector<uint8_t> h_mode;
  std::vector<int32_t> h_h0;
  mica_status_t st;
  if ((st = to_host(&h_woff, sample->win_off, n)) != MICA_OK) return st;
  if ((st = to_host(&h_wlen, sample->win_len, n)) != MICA_OK) return st;
  if ((st = to_host(&h_roff, sample->read_off, n)) != MICA_OK) return st;
  if ((st = to_host(&h_rlen, sample->read_len, n)) != MICA_OK) return st;
  if (sample->mode && (st = to_host(&h_mode, sample->mode, n)) != MICA_OK) return st;
  if (sample->ext_h0 && (st = to_host(&h_h0, sample->ext_h0, n)) != MICA_OK) return st;

  // pairs of each read-length range
  const int n_ranges = (sample->max_read_len + kRangeWidth - 1) / kRangeWidth;
  std::vector<std::vector<int64_t>> members((size_t)n_ranges);
  for (int64_t p = 0; p < n; ++p) {
    const int m = h_rlen[(size_t)p];
    if (m < 1 || m > sample->max_read_len || h_wlen[(size_t)p] < 0 || h_wlen[(size_t)p] > sample->max_win_len)
      continue;
    auto& v = members[(size_t)((m - 1) / kRangeWidth)];
    if ((int64_t)v.size() < kMaxTunePairs) v.push_back(p);
  }
  int64_t cap_n = 0;
  for (auto& v : members) cap_n = std::max<int64_t>(cap_n, (int64_t)v.size());
  if (cap_n < kMinPairs) return MICA_OK;

  const bool want_cigar = flags & MICA_OUT_CIGAR;
  const int cap = want_cigar ? std::max(sample->cigar_cap, 0) : 0;
  TuneBuffers tb;
  HIP_TRY(hipMalloc(&tb.win_off, cap_n * sizeof(uint64_t)));
  HIP_TRY(hipMalloc(&tb.win_len, cap_n * sizeof(int32_t)));
  HIP_TRY(hipMalloc(&tb.read_off, cap_n * sizeof(uint64_t)));
  HIP_TRY(hipMalloc(&tb.read_len, cap_n * sizeof(int32_t)));
  if (sample->mode) HIP_TRY(hipMalloc(&tb.mode, cap_n));
  if (sample->ext_h0) HIP_TRY(hipMalloc(&tb.ext_h0, cap_n * sizeof(int32_t)));
  HIP_TRY(hipMalloc(&tb.out, 7 * cap_n * sizeof(int32_t)));
  if (cap > 0) HIP_TRY(hipMalloc(&tb.cigar, (size_t)cap_n * cap * sizeof(uint32_t)));
  hipEvent_t e0, e1;
  HIP_TRY(hipEventCreate(&e0));
  HIP_TRY(hipEventCreate(&e1));
  struct EvGuard {
    hipEvent_t a, b;
    ~EvGuard() {
      (void)hipEventDestroy(a);
      (void)hipEventDestroy(b);
    }
  } evg{e0, e1};

  // The tuning batch: every sample pair of a tuned range, timed whole.
  // Plans of different ranges share the launch (the persistent kernels
  // balance the 16-lane classes against each other; other plans run as
  // plain launches after them), so a range's candidate is judged by the
  // time of the whole batch, one range at a time, earlier choices kept.
  std::vector<int64_t> all;
  std::vector<int> tuned;
  for (int r = 0; r < n_ranges; ++r) {
    if ((int64_t)members[(size_t)r].size() < kMinPairs) continue;
    tuned.push_back(r);
    all.insert(all.end(), members[(size_t)r].begin(), members[(size_t)r].end());
  }
  if (tuned.empty()) return MICA_OK;
  const int64_t sn = (int64_t)all.size();
  if (sn > cap_n) {
    // buffers were sized for the largest range; grow them to the whole batch
    TuneBuffers big;
    HIP_TRY(hipMalloc(&big.win_off, sn * sizeof(uint64_t)));
    HIP_TRY(hipMalloc(&big.win_len, sn * sizeof(int32_t)));
    HIP_TRY(hipMalloc(&big.read_off, sn * sizeof(uint64_t)));
    HIP_TRY(hipMalloc(&big.read_len, sn * sizeof(int32_t)));
    if (sample->mode) HIP_TRY(hipMalloc(&big.mode, sn));
    if (sample->ext_h0) HIP_TRY(hipMalloc(&big.ext_h0, sn * sizeof(int32_t)));
    HIP_TRY(hipMalloc(&big.out, 7 * sn * sizeof(int32_t)));
    if (cap > 0) HIP_TRY(hipMalloc(&big.cigar, (size_t)sn * cap * sizeof(uint32_t)));
    std::swap(tb.win_off, big.win_off);
    std::swap(tb.win_len, big.win_len);
    std::swap(tb.read_off, big.read_off);
    std::swap(tb.read_len, big.read_len);
    std::swap(tb.mode, big.mode);
    std::swap(tb.ext_h0, big.ext_h0);
    std::swap(tb.out, big.out);
    std::swap(tb.cigar, big.cigar);
  }
  if ((st = gather_up(tb.win_off, h_woff, all)) != MICA_OK) return st;
  if ((st = gather_up(tb.win_len, h_wlen, all)) != MICA_OK) return st;
  if ((st = gather_up(tb.read_off, h_roff, all)) != MICA_OK) return st;
  if ((st = gather_up(tb.read_len, h_rlen, all)) != MICA_OK) return st;
  if (sample->mode && (st = gather_up(tb.mode, h_mode, all)) != MICA_OK) return st;
  // extension start scores travel with their pairs
  if (sample->ext_h0 && (st = gather_up(tb.ext_h0, h_h0, all)) != MICA_OK) return st;
  int max_w = 0, max_m = 0, min_m = kMaxM;
  for (int64_t p : all) {
    max_w = std::max(max_w, h_wlen[(size_t)p]);
    max_m = std::max(max_m, h_rlen[(size_t)p]);
    min_m = std::min(min_m, h_rlen[(size_t)p]);
  }
  mica_batch_t sb = *sample;
  sb.win_off = tb.win_off;
  sb.win_len = tb.win_len;
  sb.read_off = tb.read_off;
  sb.read_len = tb.read_len;
  sb.mode = sample->mode ? tb.mode : nullptr;
  sb.ext_h0 = sample->ext_h0 ? tb.ext_h0 : nullptr;
  sb.n_pairs = sn;
  sb.max_read_len = max_m;
  sb.min_read_len = min_m;
  sb.max_win_len = max_w;
  sb.score = tb.out;
  sb.read_end = tb.out + sn;
  sb.ref_end = tb.out + 2 * sn;
  sb.read_start = tb.out + 3 * sn;
  sb.ref_start = tb.out + 4 * sn;
  sb.n_cigar = tb.out + 5 * sn;
  sb.status = (uint32_t*)(tb.out + 6 * sn);
  sb.cigar = tb.cigar;
  sb.cigar_cap = cap;

  // one warm-up call, then the mean of `reps` timed calls; the outputs of the
  // last call are left in the tuning buffers
  auto time_batch = [&](double* per) -> mica_status_t {
    mica_status_t e;
    if ((e = upload_plan(c)) != MICA_OK) return e;
    if ((e = mica_dp_align_batch(c, &sb, scoring, flags, stream)) != MICA_OK) return e;
    HIP_TRY(hipEventRecord(e0, stream));
    for (int k = 0; k < reps; ++k)
      if ((e = mica_dp_align_batch(c, &sb, scoring, flags, stream)) != MICA_OK) return e;
    HIP_TRY(hipEventRecord(e1, stream));
    HIP_TRY(hipEventSynchronize(e1));
    float ms = 0;
    HIP_TRY(hipEventElapsedTime(&ms, e0, e1));
    *per = (double)ms / reps;
    return MICA_OK;
  };
  auto range_lo = [](int r) { return r * kRangeWidth + 1; };
  auto range_hi = [](int r) { return std::min((r + 1) * kRangeWidth, kMaxM); };
  // reference outputs and time: the default plan on every tuned range
  for (int r : tuned)
    for (int m = range_lo(r); m <= range_hi(r); ++m) c->class_of_m[m] = (uint8_t)default_class_of(range_hi(r));
  double cur_ms = 0;
  if ((st = time_batch(&cur_ms)) != MICA_OK) return st;
  HostOutputs ref;
  if ((st = to_host(&ref.v, tb.out, 7 * sn)) != MICA_OK) return st;
  if (cap > 0 && (st = to_host(&ref.cigar, tb.cigar, sn * cap)) != MICA_OK) return st;

  int32_t written = 0;
  for (int r : tuned) {
    const int m_lo = range_lo(r), m_hi = range_hi(r);
    const std::vector<int> cands = candidates(m_hi);
    int best = cands[0], rejected = 0;
    const double before_ms = cur_ms;
    double best_ms = cur_ms;
    for (size_t ci = 1; ci < cands.size(); ++ci) {
      for (int m = m_lo; m <= m_hi; ++m) c->class_of_m[m] = (uint8_t)cands[ci];
      double per = 0;
      if ((st = time_batch(&per)) != MICA_OK) return st;
      HostOutputs got;
      if ((st = to_host(&got.v, tb.out, 7 * sn)) != MICA_OK) return st;
      if (cap > 0 && (st = to_host(&got.cigar, tb.cigar, sn * cap)) != MICA_OK) return st;
      if (!same_outputs(ref, got, sn, cap, cap > 0)) {
        ++rejected;
        continue;
      }
      // a candidate must beat the current choice by more than timing noise
      if (per < best_ms * (1.0 - kMinGain)) {
        best_ms = per;
        best = cands[ci];
      }
    }
    for (int m = m_lo; m <= m_hi; ++m) c->class_of_m[m] = (uint8_t)best;
    cur_ms = best_ms;
    if (out && written < out_cap) {
      mica_tune_entry_t& e = out[written];
      std::memset(&e, 0, sizeof(e));
      e.m_lo = m_lo;
      e.m_hi = m_hi;
      e.lanes = class_lanes(best);
      e.rows = class_rows(best);
      e.n_pairs = (int32_t)members[(size_t)r].size();
      e.n_candidates = (int32_t)cands.size();
      e.n_rejected = rejected;
      e.ms = best_ms;
      e.default_ms = before_ms;
    }
    ++written;
  }
  if ((st = upload_plan(c)) != MICA_OK) return st;
  *n_out = out ? std::min(written, out_cap) : 0;
  return MICA_OK;
}

mica_status_t mica_ctx_save_plan(mica_ctx_t c, const char* path) {
  if (!c || !path) return fail(MICA_ERR_INVALID_ARG, "NULL ctx or path");
  FILE* f = std::fopen(path, "w");
  if (!f) return fail(MICA_ERR_INVALID_ARG, std::string("cannot write ") + path);
  std::fprintf(f, "{\n  \"format\": \"mica-plan-1\",\n  \"arch\": \"%s\",\n  \"n_cu\": %d,\n  \"ranges\": [", c->arch.c_str(),
               c->n_cu);
  int m = 1;
  bool first = true;
  while (m <= kMaxM) {
    int e = m;
    while (e + 1 <= kMaxM && c->class_of_m[e + 1] == c->class_of_m[m]) ++e;
    const int cls = c->class_of_m[m];
    std::fprintf(f, "%s\n    {\"m_lo\": %d, \"m_hi\": %d, \"lanes\": %d, \"rows\": %d}", first ? "" : ",", m, e,
                 class_lanes(cls), class_rows(cls));
    first = false;
    m = e + 1;
  }
  std::fprintf(f, "\n  ]\n}\n");
  const bool ok = std::fclose(f) == 0;
  return ok ? MICA_OK : fail(MICA_ERR_INVALID_ARG, std::string("cannot write ") + path);
}

}  // extern "C"

namespace {

// Minimal reader of the plan file written above: the values of "arch",
// "n_cu" and the four integers of every object in "ranges".
struct PlanReader {
  std::string s;
  size_t pos = 0;
  bool key(const char* k, size_t from, size_t* at) const {
    const std::string q = std::string("\"") + k + "\"";
    const size_t p = s.find(q, from);
    if (p == std::string::npos) return false;
    size_t c = p + q.size();
    while (c < s.size() && std::isspace((unsigned char)s[c])) ++c;
    if (c >= s.size() || s[c] != ':') return false;
    ++c;
    while (c < s.size() && std::isspace((unsigned char)s[c])) ++c;
    *at = c;
    return true;
  }
  bool int_at(size_t at, long* v) const {
    if (at >= s.size()) return false;
    char* end = nullptr;
    *v = std::strtol(s.c_str() + at, &end, 10);
    return end != s.c_str() + at;
  }
  bool str_at(size_t at, std::string* v) const {
    if (at >= s.size() || s[at] != '"') return false;
    const size_t e = s.find('"', at + 1);
    if (e == std::string::npos) return false;
    *v = s.substr(at + 1, e - at - 1);
    return true;
  }
};

}  // namespace

extern "C" mica_status_t mica_ctx_load_plan(mica_ctx_t c, const char* path) {
  if (!c || !path) return fail(MICA_ERR_INVALID_ARG, "NULL ctx or path");
  FILE* f = std::fopen(path, "r");
  if (!f) return fail(MICA_ERR_INVALID_ARG, std::string("cannot read ") + path);
  PlanReader rd;
  char buf[4096];
  size_t got;
  while ((got = std::fread(buf, 1, sizeof(buf), f)) > 0) rd.s.append(buf, got);
  std::fclose(f);
  size_t at;
  std::string arch;
  long n_cu = 0;
  if (!rd.key("arch", 0, &at) || !rd.str_at(at, &arch) || !rd.key("n_cu", 0, &at) || !rd.int_at(at, &n_cu))
    return fail(MICA_ERR_INVALID_ARG, "plan file: missing arch or n_cu");
  if (arch != c->arch || n_cu != c->n_cu)
    return fail(MICA_ERR_INVALID_ARG, "plan file is for " + arch + " with " + std::to_string(n_cu) +
                                          " CUs, this device is " + c->arch + " with " + std::to_string(c->n_cu));
  size_t ranges;
  if (!rd.key("ranges", 0, &ranges)) return fail(MICA_ERR_INVALID_ARG, "plan file: missing ranges");
  uint8_t table[kMaxM + 1];
  std::memcpy(table, c->class_of_m, sizeof(table));
  size_t from = ranges;
  for (;;) {
    size_t a0, a1, a2, a3;
    if (!rd.key("m_lo", from, &a0)) break;
    long m_lo, m_hi, lanes, rows;
    if (!rd.int_at(a0, &m_lo) || !rd.key("m_hi", a0, &a1) || !rd.int_at(a1, &m_hi) || !rd.key("lanes", a1, &a2) ||
        !rd.int_at(a2, &lanes) || !rd.key("rows", a2, &a3) || !rd.int_at(a3, &rows))
      return fail(MICA_ERR_INVALID_ARG, "plan file: malformed range");
    const int cls = class_of((int)lanes, (int)rows);
    if (m_lo < 1 || m_hi > kMaxM || m_lo > m_hi || cls < 0 || lanes * rows < m_hi)
      return fail(MICA_ERR_INVALID_ARG, "plan file: invalid range or plan");
    for (long m = m_lo; m <= m_hi; ++m) table[m] = (uint8_t)cls;
    from = a3;
  }
  std::memcpy(c->class_of_m, table, sizeof(table));
  return upload_plan(c);
}
