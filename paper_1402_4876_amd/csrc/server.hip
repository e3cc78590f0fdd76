// Serving loop of the DP phase on one GPU: the host-side core (serve_core.h:
// queue, continuous batching over in-flight slots, replay, statistics) with
// a GPU backend per slot (its own HIP stream, library context, pinned and
// device staging), the reference resident on the device, and admission of
// device memory against the live use of all slots.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstring>
#include <memory>
#include <mutex>
#include <string>
#include <thread>
#include <vector>

#include "ctx.h"
#include "dp_common.h"
#include "mica_dp.h"
#include "serve_core.h"

using namespace mica;

namespace {

constexpr int64_t kSlotPairs = 1 << 16;         // pairs per batch
constexpr int64_t kSlotWords = kSlotPairs * 24;  // read words per batch (384 bases per read on average)
constexpr size_t kDefaultBudget = size_t(24) << 30;
constexpr int kMaxSlots = 16;
constexpr size_t kMinWorkspace = size_t(64) << 20;  // a slot's context may always grow to this

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

// Device memory of the server: a budget covering the reference, every
// slot's staging (fixed) and the slots' context workspaces (grown as
// batches need).  Before a batch, a slot's context may grow into whatever
// the budget leaves after the other slots' current allocations.
struct HbmPool {
  std::mutex mu;
  size_t budget = 0, fixed = 0;
  std::vector<size_t> held;  // per slot: its context's device workspace
  size_t grant(int s) {
    std::lock_guard<std::mutex> g(mu);
    size_t others = 0;
    for (size_t i = 0; i < held.size(); ++i)
      if ((int)i != s) others += held[i];
    const size_t left = budget > fixed + others ? budget - fixed - others : 0;
    return std::max(left, kMinWorkspace);
  }
  void record(int s, size_t bytes) {
    std::lock_guard<std::mutex> g(mu);
    held[(size_t)s] = bytes;
  }
};

class GpuSlot : public serve::Backend {
 public:
  GpuSlot(int device, int index, const uint32_t* d_ref, uint64_t ref_len, const mica_scoring_t& sc, uint32_t flags,
          int cigar_cap, HbmPool* pool)
      : device_(device), index_(index), d_ref_(d_ref), ref_len_(ref_len), sc_(sc), flags_(flags), cap_(cigar_cap),
        pool_(pool), lay_(InLayout::make()) {}
  ~GpuSlot() override {
    (void)hipSetDevice(device_);
    if (stream_) (void)hipStreamSynchronize(stream_);
    if (ctx_) mica_ctx_destroy(ctx_);
    if (done_) (void)hipEventDestroy(done_);
    if (stream_) (void)hipStreamDestroy(stream_);
    if (h_in_) (void)hipHostFree(h_in_);
    if (h_out_) (void)hipHostFree(h_out_);
    if (d_in_) (void)hipFree(d_in_);
    if (d_out_) (void)hipFree(d_out_);
  }
  static size_t out_bytes(int cap) { return align_up((size_t)7 * kSlotPairs * 4, 256) + (size_t)kSlotPairs * cap * 4; }
  static size_t staging_bytes(int cap) { return InLayout::make().total + out_bytes(cap); }

  mica_status_t init() {
    HIP_TRY(hipSetDevice(device_));
    HIP_TRY(hipStreamCreateWithFlags(&stream_, hipStreamNonBlocking));
    HIP_TRY(hipEventCreateWithFlags(&done_, hipEventDisableTiming));
    if (hipHostMalloc((void**)&h_in_, lay_.total, hipHostMallocDefault) != hipSuccess ||
        hipHostMalloc((void**)&h_out_, out_bytes(cap_), hipHostMallocDefault) != hipSuccess)
      return fail(MICA_ERR_OUT_OF_MEMORY, "cannot allocate pinned staging");
    if (hipMalloc(&d_in_, lay_.total) != hipSuccess || hipMalloc(&d_out_, out_bytes(cap_)) != hipSuccess)
      return fail(MICA_ERR_OUT_OF_MEMORY, "cannot allocate device staging");
    const mica_status_t st = mica_ctx_create(device_, kMinWorkspace, &ctx_);
    if (st != MICA_OK) return fail(st, std::string("slot context: ") + mica_last_error());
    return MICA_OK;
  }

  bool start(const serve::Batch& b, std::string* err) override {
    (void)hipSetDevice(device_);
    const InLayout& L = lay_;
    int64_t p0 = 0, w0 = 0;
    bool any_local = false;
    for (auto& r : b.reqs) {
      std::memcpy(h_in_ + L.words + (size_t)w0 * 4, r->reads.data(), r->reads.size() * 4);
      uint64_t* ro = (uint64_t*)(h_in_ + L.read_off) + p0;
      for (int64_t p = 0; p < r->n; ++p) ro[p] = r->read_off[(size_t)p] + (uint64_t)w0 * 16;
      std::memcpy((uint64_t*)(h_in_ + L.win_off) + p0, r->win_off.data(), (size_t)r->n * 8);
      std::memcpy((int32_t*)(h_in_ + L.win_len) + p0, r->win_len.data(), (size_t)r->n * 4);
      std::memcpy((int32_t*)(h_in_ + L.read_len) + p0, r->read_len.data(), (size_t)r->n * 4);
      uint8_t* md = h_in_ + L.mode + p0;
      if (r->mode.empty()) std::memset(md, 0, (size_t)r->n);
      else std::memcpy(md, r->mode.data(), (size_t)r->n);
      for (uint8_t x : r->mode) any_local |= x == 1;
      p0 += r->n;
      w0 += (int64_t)r->reads.size();
    }
    const int64_t n = p0;
    hipError_t e = hipSuccess;
    // inputs: the used prefix of each area
    auto h2d = [&](size_t off, size_t bytes) {
      if (e == hipSuccess && bytes) e = hipMemcpyAsync(d_in_ + off, h_in_ + off, bytes, hipMemcpyHostToDevice, stream_);
    };
    h2d(L.words, (size_t)w0 * 4);
    h2d(L.win_off, (size_t)n * 8);
    h2d(L.read_off, (size_t)n * 8);
    h2d(L.win_len, (size_t)n * 4);
    h2d(L.read_len, (size_t)n * 4);
    if (any_local) h2d(L.mode, (size_t)n);
    if (e != hipSuccess) {
      *err = std::string("serving H2D copy: ") + hipGetErrorString(e);
      return false;
    }
    int32_t* o = (int32_t*)d_out_;
    const size_t cig_off = align_up((size_t)7 * kSlotPairs * 4, 256);
    mica_batch_t bt;
    std::memset(&bt, 0, sizeof(bt));
    bt.ref2b = d_ref_;
    bt.ref_len = ref_len_;
    bt.win_off = (const uint64_t*)(d_in_ + L.win_off);
    bt.win_len = (const int32_t*)(d_in_ + L.win_len);
    bt.reads2b = (const uint32_t*)(d_in_ + L.words);
    bt.reads_len = (uint64_t)w0 * 16;
    bt.read_off = (const uint64_t*)(d_in_ + L.read_off);
    bt.read_len = (const int32_t*)(d_in_ + L.read_len);
    bt.mode = any_local ? (const uint8_t*)(d_in_ + L.mode) : nullptr;
    bt.default_mode = MICA_MODE_SEMIGLOBAL;
    bt.mode_mask = (1 << MICA_MODE_SEMIGLOBAL) | (1 << MICA_MODE_LOCAL);  // requests hold modes 0 and 1 only
    bt.n_pairs = n;
    bt.max_read_len = b.max_m;
    bt.max_win_len = b.max_n;
    // outputs packed at stride n so one D2H copy moves all of them
    bt.score = o;
    bt.read_end = o + n;
    bt.ref_end = o + 2 * n;
    bt.read_start = o + 3 * n;
    bt.ref_start = o + 4 * n;
    bt.n_cigar = o + 5 * n;
    bt.status = (uint32_t*)(o + 6 * n);
    bt.cigar = (uint32_t*)(d_out_ + cig_off);
    bt.cigar_cap = cap_;
    // admission of device memory: the context may grow into what the budget
    // leaves after the other slots' current workspaces
    ctx_->ws_cap = pool_->grant(index_);
    const mica_status_t st = mica_dp_align_batch(ctx_, &bt, &sc_, flags_, stream_);
    pool_->record(index_, ctx_->scratch_cap + (size_t)ctx_->pair_cap * kPairLists * 4);
    if (st != MICA_OK) {
      *err = std::string("serving batch: ") + mica_last_error();
      (void)hipStreamSynchronize(stream_);  // let what was enqueued finish before reuse
      return false;
    }
    e = hipMemcpyAsync(h_out_, d_out_, (size_t)7 * n * 4, hipMemcpyDeviceToHost, stream_);
    if (e == hipSuccess && cap_ > 0)
      e = hipMemcpyAsync(h_out_ + cig_off, d_out_ + cig_off, (size_t)n * cap_ * 4, hipMemcpyDeviceToHost, stream_);
    if (e == hipSuccess) e = hipEventRecord(done_, stream_);
    if (e != hipSuccess) {
      *err = std::string("serving D2H copy: ") + hipGetErrorString(e);
      (void)hipStreamSynchronize(stream_);
      return false;
    }
    return true;
  }

  bool finish(std::string* err) override {
    // busy slots are polled every 20 us
    hipError_t q;
    while ((q = hipEventQuery(done_)) == hipErrorNotReady) std::this_thread::sleep_for(std::chrono::microseconds(20));
    if (q != hipSuccess) {
      *err = std::string("serving event: ") + hipGetErrorString(q);
      return false;
    }
    return true;
  }

  // outputs at stride n (the pairs of the finished batch)
  const int32_t* outputs() const override { return (const int32_t*)h_out_; }
  const uint32_t* cigars() const override {
    return (const uint32_t*)(h_out_ + align_up((size_t)7 * kSlotPairs * 4, 256));
  }
  bool load_plan(const char* path, std::string* err) override {
    if (mica_ctx_load_plan(ctx_, path) == MICA_OK) return true;
    *err = mica_last_error();
    return false;
  }

 private:
  int device_, index_;
  const uint32_t* d_ref_;
  uint64_t ref_len_;
  mica_scoring_t sc_;
  uint32_t flags_;
  int cap_;
  HbmPool* pool_;
  InLayout lay_;
  hipStream_t stream_ = nullptr;
  mica_ctx_t ctx_ = nullptr;
  hipEvent_t done_ = nullptr;
  uint8_t *h_in_ = nullptr, *h_out_ = nullptr, *d_in_ = nullptr, *d_out_ = nullptr;
};

}  // namespace

struct mica_server {
  int device = 0;
  uint32_t* d_ref = nullptr;
  HbmPool pool;
  std::unique_ptr<serve::Core> core;
};

namespace {

mica_status_t core_fail(mica_status_t st, const std::string& msg) { return st == MICA_OK ? st : fail(st, msg); }

void free_server(mica_server* s) {
  s->core.reset();  // finishes queued work, joins the slot threads, frees the slots
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
  const int cap = (flags & MICA_OUT_CIGAR) ? 64 : 0;
  const size_t fixed = ref_bytes + (size_t)max_inflight_slots * GpuSlot::staging_bytes(cap);
  // every slot's context needs room for at least one block of traceback scratch
  if (fixed + (size_t)max_inflight_slots * kMinWorkspace > budget)
    return fail(MICA_ERR_OUT_OF_MEMORY, "HBM budget too small for the reference and the slots' staging");

  mica_server* s = new mica_server();
  s->device = hip_device;
  s->pool.budget = budget;
  s->pool.fixed = fixed;
  s->pool.held.assign((size_t)max_inflight_slots, 0);
  auto bail = [&](mica_status_t st, const std::string& msg) {
    free_server(s);
    return fail(st, msg);
  };
  if (hipMalloc(&s->d_ref, std::max<size_t>(ref_bytes, 256)) != hipSuccess)
    return bail(MICA_ERR_OUT_OF_MEMORY, "cannot allocate the reference");
  if (ref_len && hipMemcpy(s->d_ref, host_ref2b, (ref_len + 15) / 16 * 4, hipMemcpyHostToDevice) != hipSuccess)
    return bail(MICA_ERR_HIP, "reference upload failed");
  uint32_t bflags = flags & ~(uint32_t)MICA_SERVE_FIFO;
  if (bflags & MICA_OUT_CIGAR) bflags |= MICA_OUT_START;
  std::vector<std::unique_ptr<serve::Backend>> slots;
  for (int i = 0; i < max_inflight_slots; ++i) {
    auto g = std::make_unique<GpuSlot>(hip_device, i, s->d_ref, ref_len, *scoring, bflags, cap, &s->pool);
    const mica_status_t st = g->init();
    if (st != MICA_OK) {
      const std::string msg = mica_last_error();
      slots.clear();
      return bail(st, msg);
    }
    slots.push_back(std::move(g));
  }
  serve::Limits lim;
  lim.slot_pairs = kSlotPairs;
  lim.slot_words = kSlotWords;
  lim.cigar_cap = cap;
  lim.fifo = (flags & MICA_SERVE_FIFO) != 0;
  s->core = std::make_unique<serve::Core>(lim, std::move(slots));
  *out = s;
  return MICA_OK;
}

mica_status_t mica_server_now(mica_server_t s, double* t) {
  if (!s || !t) return fail(MICA_ERR_INVALID_ARG, "NULL argument");
  *t = s->core->now();
  return MICA_OK;
}

mica_status_t mica_server_submit(mica_server_t s, uint64_t request_id, const uint32_t* host_reads2b,
                                 const uint64_t* read_off, const int32_t* read_len, const uint64_t* win_off,
                                 const int32_t* win_len, const uint8_t* mode, int64_t n, double arrival_time_s) {
  if (!s) return fail(MICA_ERR_INVALID_ARG, "server is NULL");
  std::string err;
  const mica_status_t st =
      s->core->submit(request_id, host_reads2b, read_off, read_len, win_off, win_len, mode, n, arrival_time_s, &err);
  return core_fail(st, err);
}

mica_status_t mica_server_replay(mica_server_t s, const uint32_t* host_reads2b, const uint64_t* read_off,
                                 const int32_t* read_len, const uint64_t* win_off, const int32_t* win_len,
                                 const uint8_t* mode, const int64_t* req_first, const int64_t* req_count,
                                 const double* arrival_s, int64_t n_requests, uint64_t first_id) {
  if (!s) return fail(MICA_ERR_INVALID_ARG, "server is NULL");
  std::string err;
  const mica_status_t st = s->core->replay(host_reads2b, read_off, read_len, win_off, win_len, mode, req_first,
                                           req_count, arrival_s, n_requests, first_id, &err);
  return core_fail(st, err);
}

mica_status_t mica_server_replay_wait(mica_server_t s, double* lag_s) {
  if (!s) return fail(MICA_ERR_INVALID_ARG, "server is NULL");
  std::string err;
  const mica_status_t st = s->core->replay_wait(lag_s, &err);
  return core_fail(st, err);
}

mica_status_t mica_server_poll(mica_server_t s, uint64_t* done_ids, int64_t cap, int64_t* n_done) {
  if (!s || !n_done || cap < 0 || (cap > 0 && !done_ids)) return fail(MICA_ERR_INVALID_ARG, "bad argument");
  *n_done = s->core->poll(done_ids, cap);
  return MICA_OK;
}

mica_status_t mica_server_fetch(mica_server_t s, uint64_t request_id, int32_t* score, int32_t* read_start,
                                int32_t* read_end, int32_t* ref_start, int32_t* ref_end, uint32_t* cigar,
                                int32_t cigar_cap, int32_t* n_cigar, uint32_t* status) {
  if (!s) return fail(MICA_ERR_INVALID_ARG, "server is NULL");
  std::string err;
  const mica_status_t st = s->core->fetch(request_id, score, read_start, read_end, ref_start, ref_end, cigar,
                                          cigar_cap, n_cigar, status, &err);
  return core_fail(st, err);
}

mica_status_t mica_server_stats(mica_server_t s, double* p50_s, double* p99_s, double* gcups) {
  if (!s) return fail(MICA_ERR_INVALID_ARG, "server is NULL");
  std::string err;
  const mica_status_t st = s->core->stats(p50_s, p99_s, gcups, &err);
  return core_fail(st, err);
}

mica_status_t mica_server_load_plan(mica_server_t s, const char* path) {
  if (!s) return fail(MICA_ERR_INVALID_ARG, "server is NULL");
  std::string err;
  const mica_status_t st = s->core->load_plan(path, &err);
  return core_fail(st, err);
}

mica_status_t mica_server_reset_stats(mica_server_t s) {
  if (!s) return fail(MICA_ERR_INVALID_ARG, "server is NULL");
  s->core->reset_stats();
  return MICA_OK;
}

mica_status_t mica_server_destroy(mica_server_t s) {
  if (!s) return MICA_OK;
  (void)hipSetDevice(s->device);
  free_server(s);
  return MICA_OK;
}

}  // extern "C"
