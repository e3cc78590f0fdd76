// Serving loop of the DP phase: a resident reference on one GPU, requests of
// reads submitted from the host, continuous batching over K in-flight slots
// (each a HIP stream, a library context and pinned + device staging), and
// per-request latency statistics.
//
// This is the host side of the paper's controller design (architecture
// section: the host hands large batches to the card and keeps it busy while it
// waits on I/O), restated for one GPU: requests queue FIFO; each slot has a
// host thread that packs every queued request that fits into its staging,
// launches it on the slot's stream and hands the outputs back, so the slots'
// host work, copies and kernels all overlap.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <atomic>
#include <chrono>
#include <condition_variable>
#include <cstring>
#include <deque>
#include <memory>
#include <mutex>
#include <string>
#include <thread>
#include <unordered_map>
#include <vector>

#include "ctx.h"
#include "dp_common.h"
#include "mica_dp.h"

using namespace mica;

namespace {

constexpr int64_t kSlotPairs = 1 << 16;         // pairs per batch
constexpr int64_t kSlotWords = kSlotPairs * 24;  // read words per batch (384 bases per read on average)
constexpr size_t kDefaultBudget = size_t(24) << 30;
constexpr int kMaxSlots = 16;

double now_s(std::chrono::steady_clock::time_point t0) {
  return std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
}

struct Request {
  uint64_t id = 0;
  int64_t n = 0;
  double arrival = 0, done = 0;
  bool finished = false;
  int64_t cells = 0;
  int32_t max_m = 0, max_n = 0;
  std::vector<uint32_t> reads;  // read words, offsets rebased to the first word
  std::vector<uint64_t> read_off, win_off;
  std::vector<int32_t> read_len, win_len;
  std::vector<uint8_t> mode;
  std::vector<int32_t> out;       // 7 * n: score, read_end, ref_end, read_start, ref_start, n_cigar, status
  std::vector<uint32_t> cigar;    // the runs each read has, back to back
  std::vector<uint32_t> cig_off;  // n + 1 offsets into cigar
};

struct Slot {
  hipStream_t stream = nullptr;
  mica_ctx_t ctx = nullptr;
  hipEvent_t done = nullptr;
  uint8_t* h_in = nullptr;  // pinned: words | win_off | read_off | win_len | read_len | mode
  uint8_t* h_out = nullptr; // pinned: 7 * pairs int32 | pairs * cap cigar words
  uint8_t* d_in = nullptr;
  uint8_t* d_out = nullptr;
  size_t in_bytes = 0, out_bytes = 0;
  std::vector<std::shared_ptr<Request>> reqs;
  int64_t n_pairs = 0;
  bool busy = false;
};

// byte offsets of the staging areas of a slot
struct InLayout {
  size_t words, win_off, read_off, win_len, read_len, mode, total;
  static InLayout make() {
    InLayout l;
    size_t o = 0;
    l.words = o;
    o += align_up(kSlotWords * 4, 256);
    l.win_off = o;
    o += align_up(kSlotPairs * 8, 256);
    l.read_off = o;
    o += align_up(kSlotPairs * 8, 256);
    l.win_len = o;
    o += align_up(kSlotPairs * 4, 256);
    l.read_len = o;
    o += align_up(kSlotPairs * 4, 256);
    l.mode = o;
    o += align_up(kSlotPairs, 256);
    l.total = o;
    return l;
  }
};

}  // namespace

struct mica_server {
  int device = 0;
  mica_scoring_t scoring{};
  uint32_t flags = 0;        // mica_dp_align_batch flags
  bool fifo = false;         // one request per batch
  int cigar_cap = 0;
  uint32_t* d_ref = nullptr;
  uint64_t ref_len = 0;
  InLayout lay{};
  std::vector<Slot> slots;
  std::chrono::steady_clock::time_point t0;
  // shared state (mutex)
  std::mutex mu;
  std::condition_variable cv;
  std::deque<std::shared_ptr<Request>> queue;
  std::unordered_map<uint64_t, std::shared_ptr<Request>> live;  // submitted, not fetched
  std::deque<uint64_t> done_ids;
  std::vector<double> latencies;
  int64_t cells_done = 0;
  double first_arrival = -1, last_done = 0;
  std::string error;
  bool stop = false;
  std::vector<std::thread> workers;  // one per slot
};

namespace {

void set_error(mica_server* s, const std::string& e) {
  std::lock_guard<std::mutex> g(s->mu);
  if (s->error.empty()) s->error = e;
}

// copy a finished slot's outputs into its requests (the slot's thread owns
// them; no lock held)
void fill_outputs(mica_server* s, Slot& sl, bool failed) {
  const int64_t n = sl.n_pairs;
  const int cap = s->cigar_cap;
  const int32_t* o = (const int32_t*)sl.h_out;
  const uint32_t* cg = (const uint32_t*)(sl.h_out + align_up((size_t)7 * kSlotPairs * 4, 256));
  int64_t base = 0;
  for (auto& r : sl.reqs) {
    r->out.assign((size_t)7 * r->n, 0);
    for (int k = 0; k < 7; ++k)
      std::memcpy(r->out.data() + (size_t)k * r->n, o + (size_t)k * n + base, (size_t)r->n * 4);
    if (failed)
      for (int64_t p = 0; p < r->n; ++p) {
        r->out[(size_t)5 * r->n + p] = 0;
        r->out[(size_t)6 * r->n + p] = (int32_t)MICA_ST_INTERNAL;
      }
    if (cap > 0) {
      // keep only the runs each read has (n_cigar, at most cap), not the
      // whole cap-wide rows
      const int32_t* nc = r->out.data() + (size_t)5 * r->n;
      r->cig_off.resize((size_t)r->n + 1);
      size_t tot = 0;
      for (int64_t p = 0; p < r->n; ++p) {
        r->cig_off[(size_t)p] = (uint32_t)tot;
        const int32_t k = nc[p] < 0 ? -nc[p] : nc[p];
        tot += (size_t)std::max(0, std::min(k, cap));
      }
      r->cig_off[(size_t)r->n] = (uint32_t)tot;
      r->cigar.resize(tot);
      for (int64_t p = 0; p < r->n; ++p)
        std::memcpy(r->cigar.data() + r->cig_off[(size_t)p], cg + (size_t)(base + p) * cap,
                    (size_t)(r->cig_off[(size_t)p + 1] - r->cig_off[(size_t)p]) * 4);
    }
    base += r->n;
  }
}

// mark a slot's requests finished (lock held)
void complete_slot(mica_server* s, Slot& sl) {
  const double t = now_s(s->t0);
  for (auto& r : sl.reqs) {
    r->done = t;
    r->finished = true;
    s->latencies.push_back(r->done - r->arrival);
    s->cells_done += r->cells;
    s->done_ids.push_back(r->id);
  }
  s->last_done = std::max(s->last_done, t);
  sl.reqs.clear();
  sl.busy = false;
  sl.n_pairs = 0;
}

// pack requests into a slot and enqueue its copies and kernels (no lock held)
bool launch_slot(mica_server* s, Slot& sl) {
  const InLayout& L = s->lay;
  int64_t p0 = 0, w0 = 0;
  int32_t max_m = 0, max_n = 0;
  bool any_local = false;
  for (auto& r : sl.reqs) {
    std::memcpy(sl.h_in + L.words + (size_t)w0 * 4, r->reads.data(), r->reads.size() * 4);
    uint64_t* ro = (uint64_t*)(sl.h_in + L.read_off) + p0;
    for (int64_t p = 0; p < r->n; ++p) ro[p] = r->read_off[(size_t)p] + (uint64_t)w0 * 16;
    std::memcpy((uint64_t*)(sl.h_in + L.win_off) + p0, r->win_off.data(), (size_t)r->n * 8);
    std::memcpy((int32_t*)(sl.h_in + L.win_len) + p0, r->win_len.data(), (size_t)r->n * 4);
    std::memcpy((int32_t*)(sl.h_in + L.read_len) + p0, r->read_len.data(), (size_t)r->n * 4);
    uint8_t* md = sl.h_in + L.mode + p0;
    if (r->mode.empty()) std::memset(md, 0, (size_t)r->n);
    else std::memcpy(md, r->mode.data(), (size_t)r->n);
    for (uint8_t x : r->mode) any_local |= x == 1;
    max_m = std::max(max_m, r->max_m);
    max_n = std::max(max_n, r->max_n);
    p0 += r->n;
    w0 += (int64_t)r->reads.size();
  }
  sl.n_pairs = p0;
  const int64_t n = p0;
  hipError_t e = hipSuccess;
  // inputs: the used prefix of each area
  auto h2d = [&](size_t off, size_t bytes) {
    if (e == hipSuccess && bytes) e = hipMemcpyAsync(sl.d_in + off, sl.h_in + off, bytes, hipMemcpyHostToDevice, sl.stream);
  };
  h2d(L.words, (size_t)w0 * 4);
  h2d(L.win_off, (size_t)n * 8);
  h2d(L.read_off, (size_t)n * 8);
  h2d(L.win_len, (size_t)n * 4);
  h2d(L.read_len, (size_t)n * 4);
  if (any_local) h2d(L.mode, (size_t)n);
  if (e != hipSuccess) {
    set_error(s, std::string("serving H2D copy: ") + hipGetErrorString(e));
    return false;
  }
  int32_t* o = (int32_t*)sl.d_out;
  const size_t cig_off = align_up((size_t)7 * kSlotPairs * 4, 256);
  mica_batch_t b;
  std::memset(&b, 0, sizeof(b));
  b.ref2b = s->d_ref;
  b.ref_len = s->ref_len;
  b.win_off = (const uint64_t*)(sl.d_in + L.win_off);
  b.win_len = (const int32_t*)(sl.d_in + L.win_len);
  b.reads2b = (const uint32_t*)(sl.d_in + L.words);
  b.reads_len = (uint64_t)w0 * 16;
  b.read_off = (const uint64_t*)(sl.d_in + L.read_off);
  b.read_len = (const int32_t*)(sl.d_in + L.read_len);
  b.mode = any_local ? (const uint8_t*)(sl.d_in + L.mode) : nullptr;
  b.default_mode = MICA_MODE_SEMIGLOBAL;
  b.mode_mask = (1 << MICA_MODE_SEMIGLOBAL) | (1 << MICA_MODE_LOCAL);  // requests hold modes 0 and 1 only
  b.n_pairs = n;
  b.max_read_len = max_m;
  b.max_win_len = max_n;
  // outputs packed at stride n so one D2H copy moves all of them
  b.score = o;
  b.read_end = o + n;
  b.ref_end = o + 2 * n;
  b.read_start = o + 3 * n;
  b.ref_start = o + 4 * n;
  b.n_cigar = o + 5 * n;
  b.status = (uint32_t*)(o + 6 * n);
  b.cigar = (uint32_t*)(sl.d_out + cig_off);
  b.cigar_cap = s->cigar_cap;
  const mica_status_t st = mica_dp_align_batch(sl.ctx, &b, &s->scoring, s->flags, sl.stream);
  if (st != MICA_OK) {
    set_error(s, std::string("serving batch: ") + mica_last_error());
    return false;
  }
  e = hipMemcpyAsync(sl.h_out, sl.d_out, (size_t)7 * n * 4, hipMemcpyDeviceToHost, sl.stream);
  if (e == hipSuccess && s->cigar_cap > 0)
    e = hipMemcpyAsync(sl.h_out + cig_off, sl.d_out + cig_off, (size_t)n * s->cigar_cap * 4, hipMemcpyDeviceToHost,
                       sl.stream);
  if (e == hipSuccess) e = hipEventRecord(sl.done, sl.stream);
  if (e != hipSuccess) {
    set_error(s, std::string("serving D2H copy: ") + hipGetErrorString(e));
    return false;
  }
  return true;
}

// One thread per slot: take every queued request that fits (oldest first),
// stage and launch it on the slot's stream, wait for its event, hand the
// outputs back.  The slots' threads run their host work in parallel.
void slot_main(mica_server* s, Slot* sl) {
  (void)hipSetDevice(s->device);
  std::unique_lock<std::mutex> lk(s->mu);
  while (true) {
    if (s->queue.empty()) {
      if (s->stop) break;
      s->cv.wait_for(lk, std::chrono::milliseconds(5));
      continue;
    }
    int64_t pairs = 0, words = 0;
    while (!s->queue.empty()) {
      const auto& r = s->queue.front();
      if (pairs + r->n > kSlotPairs || words + (int64_t)r->reads.size() > kSlotWords) break;
      pairs += r->n;
      words += (int64_t)r->reads.size();
      sl->reqs.push_back(r);
      s->queue.pop_front();
      if (s->fifo) break;
    }
    sl->busy = true;
    lk.unlock();
    bool ok = launch_slot(s, *sl);
    if (ok) {
      // busy slots are polled every 20 us
      hipError_t q;
      while ((q = hipEventQuery(sl->done)) == hipErrorNotReady) std::this_thread::sleep_for(std::chrono::microseconds(20));
      if (q != hipSuccess) {
        set_error(s, std::string("serving event: ") + hipGetErrorString(q));
        ok = false;
      }
    } else {
      (void)hipStreamSynchronize(sl->stream);  // let what was enqueued finish before reuse
    }
    fill_outputs(s, *sl, !ok);
    lk.lock();
    complete_slot(s, *sl);
  }
}

void free_server(mica_server* s) {
  for (Slot& sl : s->slots) {
    if (sl.ctx) mica_ctx_destroy(sl.ctx);
    if (sl.done) (void)hipEventDestroy(sl.done);
    if (sl.stream) (void)hipStreamDestroy(sl.stream);
    if (sl.h_in) (void)hipHostFree(sl.h_in);
    if (sl.h_out) (void)hipHostFree(sl.h_out);
    if (sl.d_in) (void)hipFree(sl.d_in);
    if (sl.d_out) (void)hipFree(sl.d_out);
  }
  if (s->d_ref) (void)hipFree(s->d_ref);
  delete s;
}

}  // namespace

extern "C" {

mica_status_t mica_server_create(int hip_device, const uint32_t* host_ref2b, uint64_t ref_len, size_t hbm_budget_bytes,
                                 int max_inflight_slots, const mica_scoring_t* scoring, uint32_t flags,
                                 mica_server_t* out) {
  if (!out || !scoring || (!host_ref2b && ref_len)) return fail(MICA_ERR_INVALID_ARG, "NULL argument");
  *out = nullptr;
  if (max_inflight_slots < 1 || max_inflight_slots > kMaxSlots)
    return fail(MICA_ERR_INVALID_ARG, "max_inflight_slots must be in 1..16");
  const uint32_t known = MICA_OUT_START | MICA_OUT_CIGAR | MICA_FORCE_INT32 | MICA_PLAIN_LAUNCH | MICA_NO_GRAPH |
                         MICA_SERVE_FIFO;
  if (flags & ~known) return fail(MICA_ERR_INVALID_ARG, "unknown flag bits");
  if (scoring->match < 1 || scoring->match > 4096 || scoring->mismatch > 0 || scoring->mismatch < -4096 ||
      scoring->gap_open < 0 || scoring->gap_open > 4096 || scoring->gap_extend < 1 || scoring->gap_extend > 4096)
    return fail(MICA_ERR_INVALID_ARG, "scoring outside the supported range");
  int ndev = 0;
  HIP_TRY(hipGetDeviceCount(&ndev));
  if (hip_device < 0 || hip_device >= ndev) return fail(MICA_ERR_INVALID_ARG, "no such HIP device");
  HIP_TRY(hipSetDevice(hip_device));
  const size_t budget = hbm_budget_bytes ? hbm_budget_bytes : kDefaultBudget;
  const size_t ref_bytes = align_up((ref_len + 15) / 16 * 4, 256);
  const InLayout lay = InLayout::make();
  const int cap = (flags & MICA_OUT_CIGAR) ? 64 : 0;
  const size_t out_bytes = align_up((size_t)7 * kSlotPairs * 4, 256) + (size_t)kSlotPairs * cap * 4;
  const size_t per_slot_fixed = lay.total + out_bytes;
  const size_t fixed = ref_bytes + (size_t)max_inflight_slots * per_slot_fixed;
  // every slot's context needs room for at least one block of traceback scratch
  const size_t min_ws = size_t(64) << 20;
  if (fixed + (size_t)max_inflight_slots * min_ws > budget)
    return fail(MICA_ERR_OUT_OF_MEMORY, "HBM budget too small for the reference and the slots' staging");
  const size_t ws = (budget - fixed) / (size_t)max_inflight_slots;

  mica_server* s = new mica_server();
  s->device = hip_device;
  s->scoring = *scoring;
  s->fifo = flags & MICA_SERVE_FIFO;
  s->flags = flags & ~(uint32_t)MICA_SERVE_FIFO;
  if (s->flags & MICA_OUT_CIGAR) s->flags |= MICA_OUT_START;
  s->cigar_cap = cap;
  s->ref_len = ref_len;
  s->lay = lay;
  s->t0 = std::chrono::steady_clock::now();
  auto bail = [&](mica_status_t st, const std::string& msg) {
    free_server(s);
    return fail(st, msg);
  };
  if (hipMalloc(&s->d_ref, std::max<size_t>(ref_bytes, 256)) != hipSuccess)
    return bail(MICA_ERR_OUT_OF_MEMORY, "cannot allocate the reference");
  if (ref_len && hipMemcpy(s->d_ref, host_ref2b, (ref_len + 15) / 16 * 4, hipMemcpyHostToDevice) != hipSuccess)
    return bail(MICA_ERR_HIP, "reference upload failed");
  s->slots.resize((size_t)max_inflight_slots);
  for (Slot& sl : s->slots) {
    sl.in_bytes = lay.total;
    sl.out_bytes = out_bytes;
    if (hipStreamCreateWithFlags(&sl.stream, hipStreamNonBlocking) != hipSuccess ||
        hipEventCreateWithFlags(&sl.done, hipEventDisableTiming) != hipSuccess)
      return bail(MICA_ERR_HIP, "cannot create slot stream / event");
    if (hipHostMalloc((void**)&sl.h_in, lay.total, hipHostMallocDefault) != hipSuccess ||
        hipHostMalloc((void**)&sl.h_out, out_bytes, hipHostMallocDefault) != hipSuccess)
      return bail(MICA_ERR_OUT_OF_MEMORY, "cannot allocate pinned staging");
    if (hipMalloc(&sl.d_in, lay.total) != hipSuccess || hipMalloc(&sl.d_out, out_bytes) != hipSuccess)
      return bail(MICA_ERR_OUT_OF_MEMORY, "cannot allocate device staging");
    const mica_status_t st = mica_ctx_create(hip_device, ws, &sl.ctx);
    if (st != MICA_OK) return bail(st, std::string("slot context: ") + mica_last_error());
  }
  for (Slot& sl : s->slots) s->workers.emplace_back(slot_main, s, &sl);
  *out = s;
  return MICA_OK;
}

mica_status_t mica_server_now(mica_server_t s, double* t) {
  if (!s || !t) return fail(MICA_ERR_INVALID_ARG, "NULL argument");
  *t = now_s(s->t0);
  return MICA_OK;
}

mica_status_t mica_server_submit(mica_server_t s, uint64_t request_id, const uint32_t* host_reads2b,
                                 const uint64_t* read_off, const int32_t* read_len, const uint64_t* win_off,
                                 const int32_t* win_len, const uint8_t* mode, int64_t n, double arrival_time_s) {
  if (!s) return fail(MICA_ERR_INVALID_ARG, "server is NULL");
  if (n < 0) return fail(MICA_ERR_INVALID_ARG, "n < 0");
  if (n > 0 && (!host_reads2b || !read_off || !read_len || !win_off || !win_len))
    return fail(MICA_ERR_INVALID_ARG, "NULL request array");
  if (n > kSlotPairs) return fail(MICA_ERR_LIMIT, "request larger than one serving batch (65,536 reads)");
  auto r = std::make_shared<Request>();
  r->id = request_id;
  r->n = n;
  uint64_t lo = UINT64_MAX, hi = 0;
  for (int64_t p = 0; p < n; ++p) {
    if (read_len[p] < 0 || win_len[p] < 0) return fail(MICA_ERR_INVALID_ARG, "negative length");
    if (read_len[p] > kMaxM || win_len[p] > kMaxN) return fail(MICA_ERR_LIMIT, "read or window over the library limits");
    lo = std::min(lo, read_off[p]);
    hi = std::max(hi, read_off[p] + (uint64_t)read_len[p]);
    if (mode && mode[p] > 1) return fail(MICA_ERR_INVALID_ARG, "mode must be 0 or 1");
    r->max_m = std::max(r->max_m, read_len[p]);
    r->max_n = std::max(r->max_n, win_len[p]);
    r->cells += (int64_t)read_len[p] * win_len[p];
  }
  const uint64_t w_lo = n ? lo / 16 : 0, w_hi = n ? (hi + 15) / 16 : 0;
  if ((int64_t)(w_hi - w_lo) > kSlotWords) return fail(MICA_ERR_LIMIT, "request reads larger than one serving batch");
  r->reads.assign(host_reads2b + w_lo, host_reads2b + w_hi);
  r->read_off.resize((size_t)n);
  for (int64_t p = 0; p < n; ++p) r->read_off[(size_t)p] = read_off[p] - w_lo * 16;
  r->win_off.assign(win_off, win_off + n);
  r->read_len.assign(read_len, read_len + n);
  r->win_len.assign(win_len, win_len + n);
  if (mode) r->mode.assign(mode, mode + n);
  {
    std::lock_guard<std::mutex> g(s->mu);
    if (s->stop) return fail(MICA_ERR_BUSY, "server is shutting down");
    if (s->live.count(request_id)) return fail(MICA_ERR_INVALID_ARG, "request id already in use");
    r->arrival = arrival_time_s >= 0 ? arrival_time_s : now_s(s->t0);
    if (s->first_arrival < 0 || r->arrival < s->first_arrival) s->first_arrival = r->arrival;
    s->live.emplace(request_id, r);
    s->queue.push_back(r);
  }
  s->cv.notify_one();
  return MICA_OK;
}

mica_status_t mica_server_poll(mica_server_t s, uint64_t* done_ids, int64_t cap, int64_t* n_done) {
  if (!s || !n_done || cap < 0 || (cap > 0 && !done_ids)) return fail(MICA_ERR_INVALID_ARG, "bad argument");
  std::lock_guard<std::mutex> g(s->mu);
  int64_t k = 0;
  while (k < cap && !s->done_ids.empty()) {
    done_ids[k++] = s->done_ids.front();
    s->done_ids.pop_front();
  }
  *n_done = k;
  return MICA_OK;
}

mica_status_t mica_server_fetch(mica_server_t s, uint64_t request_id, int32_t* score, int32_t* read_start,
                                int32_t* read_end, int32_t* ref_start, int32_t* ref_end, uint32_t* cigar,
                                int32_t cigar_cap, int32_t* n_cigar, uint32_t* status) {
  if (!s) return fail(MICA_ERR_INVALID_ARG, "server is NULL");
  std::shared_ptr<Request> r;
  {
    std::lock_guard<std::mutex> g(s->mu);
    auto it = s->live.find(request_id);
    if (it == s->live.end()) return fail(MICA_ERR_INVALID_ARG, "unknown request id");
    if (!it->second->finished) return fail(MICA_ERR_BUSY, "request not finished");
    r = it->second;
    s->live.erase(it);
  }
  const int64_t n = r->n;
  const int32_t* o = r->out.data();
  auto put = [&](int32_t* dst, int k) {
    if (dst) std::memcpy(dst, o + (size_t)k * n, (size_t)n * 4);
  };
  put(score, 0);
  put(read_end, 1);
  put(ref_end, 2);
  put(read_start, 3);
  put(ref_start, 4);
  put(n_cigar, 5);
  put((int32_t*)status, 6);
  if (cigar && cigar_cap > 0 && s->cigar_cap > 0 && !r->cig_off.empty()) {
    // the runs of each read (words past them in a row are left as they were)
    for (int64_t p = 0; p < n; ++p) {
      const uint32_t a = r->cig_off[(size_t)p];
      const uint32_t k = std::min<uint32_t>(r->cig_off[(size_t)p + 1] - a, (uint32_t)cigar_cap);
      std::memcpy(cigar + (size_t)p * cigar_cap, r->cigar.data() + a, (size_t)k * 4);
    }
  }
  return MICA_OK;
}

mica_status_t mica_server_stats(mica_server_t s, double* p50_s, double* p99_s, double* gcups) {
  if (!s) return fail(MICA_ERR_INVALID_ARG, "server is NULL");
  std::lock_guard<std::mutex> g(s->mu);
  if (!s->error.empty()) return fail(MICA_ERR_HIP, s->error);
  std::vector<double> v = s->latencies;
  auto pct = [&](double q) {
    if (v.empty()) return 0.0;
    const size_t k = std::min(v.size() - 1, (size_t)(q * (double)(v.size() - 1) + 0.5));
    std::nth_element(v.begin(), v.begin() + (ptrdiff_t)k, v.end());
    return v[k];
  };
  if (p50_s) *p50_s = pct(0.50);
  if (p99_s) *p99_s = pct(0.99);
  if (gcups) {
    const double span = s->last_done - std::max(s->first_arrival, 0.0);
    *gcups = span > 0 ? (double)s->cells_done / span / 1e9 : 0.0;
  }
  return MICA_OK;
}

mica_status_t mica_server_reset_stats(mica_server_t s) {
  if (!s) return fail(MICA_ERR_INVALID_ARG, "server is NULL");
  std::lock_guard<std::mutex> g(s->mu);
  s->latencies.clear();
  s->cells_done = 0;
  s->first_arrival = -1;
  s->last_done = 0;
  return MICA_OK;
}

mica_status_t mica_server_destroy(mica_server_t s) {
  if (!s) return MICA_OK;
  {
    std::lock_guard<std::mutex> g(s->mu);
    s->stop = true;
  }
  s->cv.notify_all();
  for (auto& w : s->workers)
    if (w.joinable()) w.join();
  (void)hipSetDevice(s->device);
  for (Slot& sl : s->slots)
    if (sl.stream) (void)hipStreamSynchronize(sl.stream);
  free_server(s);
  return MICA_OK;
}

}  // extern "C"
