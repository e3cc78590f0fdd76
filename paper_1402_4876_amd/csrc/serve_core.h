// Host side of the serving loop, independent of the GPU: the request queue,
// packing of queued requests into in-flight slots (continuous batching),
// hand-back of each request's outputs, the replay of a request schedule and
// latency statistics.  A slot runs its batches on a Backend: the GPU (the
// library's server) or a test double that computes on the host with injected
// delays (the tests' check of admission, ordering and slot reuse).
//
// This is the host controller of the paper's design (Methods, architecture
// & parallelism: the host hands the card large batches and keeps it busy
// while it waits), restated for one GPU and a request stream.
#pragma once

#include <algorithm>
#include <atomic>
#include <chrono>
#include <condition_variable>
#include <cstdint>
#include <cstring>
#include <deque>
#include <memory>
#include <mutex>
#include <string>
#include <thread>
#include <unordered_map>
#include <vector>

#include "mica_dp.h"

namespace mica {
namespace serve {

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

// The requests one slot runs together, in queue order.
struct Batch {
  std::vector<std::shared_ptr<Request>> reqs;
  int64_t n_pairs = 0, n_words = 0;
  int32_t max_m = 0, max_n = 0;
};

// What a slot runs its batches on.  start() stages the batch's inputs and
// launches it; finish() waits for it; the outputs of a finished batch are
// 7 arrays of n_pairs int32 at stride n_pairs (score, read_end, ref_end,
// read_start, ref_start, n_cigar, status) and cigar_cap words per pair.
class Backend {
 public:
  virtual ~Backend() = default;
  virtual bool start(const Batch& b, std::string* err) = 0;
  virtual bool finish(std::string* err) = 0;
  virtual const int32_t* outputs() const = 0;
  virtual const uint32_t* cigars() const = 0;
  // Take a plan file (the library's per-read-length kernel plan) for the
  // slot's later batches; called only while the slot is idle.
  virtual bool load_plan(const char* path, std::string* err) {
    (void)path;
    (void)err;
    return true;
  }
};

struct Limits {
  int64_t slot_pairs = 1 << 16;  // pairs per batch
  int64_t slot_words = (1 << 16) * 24;  // read words per batch
  int cigar_cap = 0;             // CIGAR runs kept per read (0: no CIGAR)
  bool fifo = false;             // one request per batch
};

inline double now_s(std::chrono::steady_clock::time_point t0) {
  return std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
}

class Core {
 public:
  Core(const Limits& lim, std::vector<std::unique_ptr<Backend>> slots)
      : lim_(lim), backends_(std::move(slots)), t0_(std::chrono::steady_clock::now()) {
    slot_busy_.assign(backends_.size(), 0);
    batches_run_.assign(backends_.size(), 0);
    for (size_t i = 0; i < backends_.size(); ++i) workers_.emplace_back(&Core::slot_main, this, (int)i);
  }
  ~Core() { stop(); }

  // Finish the queued work and join the slot threads (and a replay).
  void stop() {
    replay_wait(nullptr);
    {
      std::lock_guard<std::mutex> g(mu_);
      stop_ = true;
    }
    cv_.notify_all();
    for (auto& w : workers_)
      if (w.joinable()) w.join();
    workers_.clear();
  }

  double now() const { return now_s(t0_); }
  const Limits& limits() const { return lim_; }

  // Load a plan file into every slot once the queued and running batches
  // have finished; submissions wait meanwhile (the lock is held throughout).
  mica_status_t load_plan(const char* path, std::string* err) {
    if (!path) return set(err, MICA_ERR_INVALID_ARG, "NULL plan path");
    std::unique_lock<std::mutex> lk(mu_);
    idle_cv_.wait(lk, [this] {
      if (!queue_.empty()) return false;
      for (char b : slot_busy_)
        if (b) return false;
      return true;
    });
    for (auto& be : backends_)
      if (!be->load_plan(path, err)) return MICA_ERR_INVALID_ARG;
    ++plans_loaded_;
    return MICA_OK;
  }
  int64_t plans_loaded() {
    std::lock_guard<std::mutex> g(mu_);
    return plans_loaded_;
  }

  // Validate and copy a request into the queue.  Returns MICA_OK or an error
  // with its text in *err.
  mica_status_t submit(uint64_t id, const uint32_t* reads2b, const uint64_t* read_off, const int32_t* read_len,
                       const uint64_t* win_off, const int32_t* win_len, const uint8_t* mode, int64_t n,
                       double arrival, std::string* err) {
    if (n < 0) return set(err, MICA_ERR_INVALID_ARG, "n < 0");
    if (n > 0 && (!reads2b || !read_off || !read_len || !win_off || !win_len))
      return set(err, MICA_ERR_INVALID_ARG, "NULL request array");
    if (n > lim_.slot_pairs) return set(err, MICA_ERR_LIMIT, "request larger than one serving batch (65,536 reads)");
    auto r = std::make_shared<Request>();
    r->id = id;
    r->n = n;
    uint64_t lo = UINT64_MAX, hi = 0;
    for (int64_t p = 0; p < n; ++p) {
      if (read_len[p] < 0 || win_len[p] < 0) return set(err, MICA_ERR_INVALID_ARG, "negative length");
      if (read_len[p] > MICA_MAX_READ_LEN || win_len[p] > MICA_MAX_WIN_LEN)
        return set(err, MICA_ERR_LIMIT, "read or window over the library limits");
      if (mode && mode[p] > 1) return set(err, MICA_ERR_INVALID_ARG, "mode must be 0 or 1");
      lo = std::min(lo, read_off[p]);
      hi = std::max(hi, read_off[p] + (uint64_t)read_len[p]);
      r->max_m = std::max(r->max_m, read_len[p]);
      r->max_n = std::max(r->max_n, win_len[p]);
      r->cells += (int64_t)read_len[p] * win_len[p];
    }
    const uint64_t w_lo = n ? lo / 16 : 0, w_hi = n ? (hi + 15) / 16 : 0;
    if ((int64_t)(w_hi - w_lo) > lim_.slot_words)
      return set(err, MICA_ERR_LIMIT, "request reads larger than one serving batch");
    r->reads.assign(reads2b + w_lo, reads2b + w_hi);
    r->read_off.resize((size_t)n);
    for (int64_t p = 0; p < n; ++p) r->read_off[(size_t)p] = read_off[p] - w_lo * 16;
    r->win_off.assign(win_off, win_off + n);
    r->read_len.assign(read_len, read_len + n);
    r->win_len.assign(win_len, win_len + n);
    if (mode) r->mode.assign(mode, mode + n);
    {
      std::lock_guard<std::mutex> g(mu_);
      if (stop_) return set(err, MICA_ERR_BUSY, "server is shutting down");
      if (live_.count(id)) return set(err, MICA_ERR_INVALID_ARG, "request id already in use");
      r->arrival = arrival >= 0 ? arrival : now();
      if (first_arrival_ < 0 || r->arrival < first_arrival_) first_arrival_ = r->arrival;
      live_.emplace(id, r);
      queue_.push_back(r);
    }
    cv_.notify_one();
    return MICA_OK;
  }

  int64_t poll(uint64_t* ids, int64_t cap) {
    std::lock_guard<std::mutex> g(mu_);
    int64_t k = 0;
    while (k < cap && !done_ids_.empty()) {
      ids[k++] = done_ids_.front();
      done_ids_.pop_front();
    }
    return k;
  }

  // A finished request's outputs (NULL pointers skip an output); the request
  // is forgotten.
  mica_status_t fetch(uint64_t id, int32_t* score, int32_t* read_start, int32_t* read_end, int32_t* ref_start,
                      int32_t* ref_end, uint32_t* cigar, int32_t cigar_cap, int32_t* n_cigar, uint32_t* status,
                      std::string* err) {
    std::shared_ptr<Request> r;
    {
      std::lock_guard<std::mutex> g(mu_);
      auto it = live_.find(id);
      if (it == live_.end()) return set(err, MICA_ERR_INVALID_ARG, "unknown request id");
      if (!it->second->finished) return set(err, MICA_ERR_BUSY, "request not finished");
      r = it->second;
      live_.erase(it);
    }
    const int64_t n = r->n;
    const int32_t* o = r->out.data();
    auto put = [&](int32_t* dst, int k) {
      if (dst && n) std::memcpy(dst, o + (size_t)k * n, (size_t)n * 4);
    };
    put(score, 0);
    put(read_end, 1);
    put(ref_end, 2);
    put(read_start, 3);
    put(ref_start, 4);
    put(n_cigar, 5);
    put((int32_t*)status, 6);
    if (cigar && cigar_cap > 0 && lim_.cigar_cap > 0 && !r->cig_off.empty()) {
      // the runs of each read (words past them in a row are left as they were)
      for (int64_t p = 0; p < n; ++p) {
        const uint32_t a = r->cig_off[(size_t)p];
        const uint32_t k = std::min<uint32_t>(r->cig_off[(size_t)p + 1] - a, (uint32_t)cigar_cap);
        if (k) std::memcpy(cigar + (size_t)p * cigar_cap, r->cigar.data() + a, (size_t)k * 4);
      }
    }
    return MICA_OK;
  }

  mica_status_t stats(double* p50, double* p99, double* gcups, std::string* err) {
    std::lock_guard<std::mutex> g(mu_);
    if (!error_.empty()) return set(err, MICA_ERR_HIP, error_);
    std::vector<double> v = latencies_;
    auto pct = [&](double q) {
      if (v.empty()) return 0.0;
      const size_t k = std::min(v.size() - 1, (size_t)(q * (double)(v.size() - 1) + 0.5));
      std::nth_element(v.begin(), v.begin() + (ptrdiff_t)k, v.end());
      return v[k];
    };
    if (p50) *p50 = pct(0.50);
    if (p99) *p99 = pct(0.99);
    if (gcups) {
      const double span = last_done_ - std::max(first_arrival_, 0.0);
      *gcups = span > 0 ? (double)cells_done_ / span / 1e9 : 0.0;
    }
    return MICA_OK;
  }

  void reset_stats() {
    std::lock_guard<std::mutex> g(mu_);
    latencies_.clear();
    cells_done_ = 0;
    first_arrival_ = -1;
    last_done_ = 0;
  }

  // batches each slot has run (the test double checks slot reuse)
  std::vector<int64_t> batches_run() {
    std::lock_guard<std::mutex> g(mu_);
    return batches_run_;
  }

  void set_error(const std::string& e) {
    std::lock_guard<std::mutex> g(mu_);
    if (error_.empty()) error_ = e;
  }

  // Replay a request schedule from a host thread of its own: request r is
  // reads [first[r], first[r] + count[r]) of the given arrays, submitted
  // with id first_id + r at server time arrival[r] (sleeping until then).
  // The arrays must stay valid until replay_wait returns.
  mica_status_t replay(const uint32_t* reads2b, const uint64_t* read_off, const int32_t* read_len,
                       const uint64_t* win_off, const int32_t* win_len, const uint8_t* mode, const int64_t* first,
                       const int64_t* count, const double* arrival, int64_t n_req, uint64_t first_id,
                       std::string* err) {
    if (n_req < 0 || (n_req > 0 && (!first || !count || !arrival)))
      return set(err, MICA_ERR_INVALID_ARG, "bad replay schedule");
    if (replayer_.joinable()) return set(err, MICA_ERR_BUSY, "a replay is already running");
    replay_lag_ = 0;
    replay_status_ = MICA_OK;
    replay_error_.clear();
    replayer_ = std::thread([=]() {
      double lag = 0;
      for (int64_t r = 0; r < n_req; ++r) {
        double t = now();
        while (arrival[r] > t) {
          const double dt = arrival[r] - t;
          if (dt > 0.0004) std::this_thread::sleep_for(std::chrono::duration<double>(dt - 0.0003));
          t = now();
        }
        lag = std::max(lag, t - arrival[r]);
        const int64_t f = first[r];
        std::string e;
        const mica_status_t st =
            submit(first_id + (uint64_t)r, reads2b, read_off + f, read_len + f, win_off + f, win_len + f,
                   mode ? mode + f : nullptr, count[r], arrival[r], &e);
        if (st != MICA_OK && replay_status_ == MICA_OK) {
          replay_status_ = st;
          replay_error_ = e;
        }
      }
      replay_lag_ = lag;
    });
    return MICA_OK;
  }

  // Wait for the replay thread; *lag = how far the latest submission ran
  // behind its scheduled arrival (seconds).
  mica_status_t replay_wait(double* lag, std::string* err = nullptr) {
    if (replayer_.joinable()) replayer_.join();
    if (lag) *lag = replay_lag_;
    if (replay_status_ != MICA_OK) return set(err, replay_status_, "replayed request: " + replay_error_);
    return MICA_OK;
  }

 private:
  static mica_status_t set(std::string* err, mica_status_t st, const std::string& msg) {
    if (err) *err = msg;
    return st;
  }

  // copy a finished batch's outputs into its requests (no lock held)
  void hand_back(const Batch& b, const Backend& be, bool failed) {
    const int64_t n = b.n_pairs;
    const int cap = lim_.cigar_cap;
    const int32_t* o = be.outputs();
    const uint32_t* cg = be.cigars();
    int64_t base = 0;
    for (auto& r : b.reqs) {
      r->out.assign((size_t)7 * r->n, 0);
      if (!failed)
        for (int k = 0; k < 7; ++k)
          if (r->n) std::memcpy(r->out.data() + (size_t)k * r->n, o + (size_t)k * n + base, (size_t)r->n * 4);
      if (failed)
        for (int64_t p = 0; p < r->n; ++p) r->out[(size_t)6 * r->n + p] = (int32_t)MICA_ST_INTERNAL;
      if (cap > 0) {
        // keep only the runs each read has (n_cigar, at most cap), not the
        // whole cap-wide rows
        const int32_t* nc = r->out.data() + (size_t)5 * r->n;
        r->cig_off.resize((size_t)r->n + 1);
        size_t tot = 0;
        for (int64_t p = 0; p < r->n; ++p) {
          r->cig_off[(size_t)p] = (uint32_t)tot;
          const int32_t k = nc[p] < 0 ? -nc[p] : nc[p];
          tot += failed ? 0 : (size_t)std::max(0, std::min(k, cap));
        }
        r->cig_off[(size_t)r->n] = (uint32_t)tot;
        r->cigar.resize(tot);
        for (int64_t p = 0; p < r->n; ++p)
          if (r->cig_off[(size_t)p + 1] > r->cig_off[(size_t)p])
            std::memcpy(r->cigar.data() + r->cig_off[(size_t)p], cg + (size_t)(base + p) * cap,
                        (size_t)(r->cig_off[(size_t)p + 1] - r->cig_off[(size_t)p]) * 4);
      }
      base += r->n;
    }
  }

  // One thread per slot: take every queued request that fits (oldest first),
  // run the batch on the slot's backend, hand each request its outputs.
  void slot_main(int s) {
    Backend& be = *backends_[(size_t)s];
    std::unique_lock<std::mutex> lk(mu_);
    while (true) {
      // woken by a submission, by stop(), or by a slot that left work queued
      cv_.wait(lk, [this] { return !queue_.empty() || stop_; });
      if (queue_.empty()) break;  // stopping, nothing left
      Batch b;
      while (!queue_.empty()) {
        const auto& r = queue_.front();
        if (b.n_pairs + r->n > lim_.slot_pairs || b.n_words + (int64_t)r->reads.size() > lim_.slot_words) break;
        b.n_pairs += r->n;
        b.n_words += (int64_t)r->reads.size();
        b.max_m = std::max(b.max_m, r->max_m);
        b.max_n = std::max(b.max_n, r->max_n);
        b.reqs.push_back(r);
        queue_.pop_front();
        if (lim_.fifo) break;
      }
      slot_busy_[(size_t)s] = 1;
      const bool more = !queue_.empty();
      lk.unlock();
      if (more) cv_.notify_one();  // what did not fit goes to another slot
      std::string e;
      bool ok = be.start(b, &e);
      if (ok) ok = be.finish(&e);
      if (!ok) set_error(e);
      hand_back(b, be, !ok);
      lk.lock();
      const double t = now();
      for (auto& r : b.reqs) {
        r->done = t;
        r->finished = true;
        latencies_.push_back(r->done - r->arrival);
        cells_done_ += r->cells;
        done_ids_.push_back(r->id);
      }
      last_done_ = std::max(last_done_, t);
      slot_busy_[(size_t)s] = 0;
      batches_run_[(size_t)s]++;
      idle_cv_.notify_all();
    }
  }

  Limits lim_;
  std::vector<std::unique_ptr<Backend>> backends_;
  std::chrono::steady_clock::time_point t0_;
  std::mutex mu_;
  std::condition_variable cv_;
  std::condition_variable idle_cv_;  // a slot finished a batch
  int64_t plans_loaded_ = 0;
  std::deque<std::shared_ptr<Request>> queue_;
  std::unordered_map<uint64_t, std::shared_ptr<Request>> live_;  // submitted, not fetched
  std::deque<uint64_t> done_ids_;
  std::vector<double> latencies_;
  std::vector<char> slot_busy_;
  std::vector<int64_t> batches_run_;
  int64_t cells_done_ = 0;
  double first_arrival_ = -1, last_done_ = 0;
  std::string error_;
  bool stop_ = false;
  std::vector<std::thread> workers_;
  std::thread replayer_;
  std::atomic<double> replay_lag_{0};
  mica_status_t replay_status_ = MICA_OK;
  std::string replay_error_;
};

}  // namespace serve
}  // namespace mica
