// Host test double of the serving loop: the serving core of the library
// (paper_1402_4876_amd/csrc/serve_core.h, the same queue, batching, slot
// threads, hand-back, replay and statistics the GPU server runs) driven with
// slots that compute on the host with the CPU oracle and injected delays.
// Checks that every request gets exactly its own results (equal to the oracle
// on that request alone), that batches respect the slot limits and take
// requests in queue order, that slots are reused, that the FIFO mode runs one
// request per batch, that a failing batch marks its requests and reports the
// error, that replayed schedules are submitted on time, and that stopping
// finishes the queued work.  Built and run by tests/test_serve_double.py,
// with AddressSanitizer and UndefinedBehaviorSanitizer, and with
// ThreadSanitizer.  Exit status 0 = every check passed.
#include <atomic>
#include <chrono>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <mutex>
#include <random>
#include <set>
#include <thread>
#include <vector>

#include "serve_core.h"

extern "C" int oracle_align_batch(const uint8_t* ref, int64_t ref_len, const int64_t* win_off,
                                  const int32_t* win_len, const uint8_t* reads, int64_t reads_len,
                                  const int64_t* read_off, const int32_t* read_len, const uint8_t* mode,
                                  int32_t default_mode, int64_t n_pairs, int32_t match, int32_t mismatch,
                                  int32_t gap_open, int32_t gap_extend, int32_t want_trace, int32_t cigar_cap,
                                  int32_t* score, int32_t* read_start, int32_t* read_end, int32_t* ref_start,
                                  int32_t* ref_end, uint32_t* cigar, int32_t* n_cigar, uint32_t* status,
                                  int32_t n_threads);

using namespace mica::serve;

static int g_failures = 0;
#define CHECK(cond, ...)                                   \
  do {                                                     \
    if (!(cond)) {                                         \
      std::fprintf(stderr, "CHECK failed (%s:%d) %s: ", __FILE__, __LINE__, #cond); \
      std::fprintf(stderr, __VA_ARGS__);                   \
      std::fprintf(stderr, "\n");                          \
      ++g_failures;                                        \
    }                                                      \
  } while (0)

constexpr int kCap = 16;

struct World {
  std::vector<uint8_t> ref;      // reference codes
  std::vector<uint8_t> reads;    // read codes, back to back
  std::vector<uint32_t> words;   // the same reads, 2-bit packed
  std::vector<uint64_t> read_off, win_off;
  std::vector<int32_t> read_len, win_len;
  std::vector<uint8_t> mode;
};

static World make_world(int n_reads, uint32_t seed) {
  std::mt19937 rng(seed);
  World w;
  w.ref.resize(20000);
  for (auto& c : w.ref) c = (uint8_t)(rng() & 3);
  uint64_t pos = 0;
  for (int k = 0; k < n_reads; ++k) {
    const int m = (int)(rng() % 40);  // 0..39 bases, some empty
    const int n = (int)(rng() % 60);
    const uint64_t wo = rng() % (w.ref.size() - 64);
    pos += rng() % 5;  // unaligned read offsets
    w.read_off.push_back(pos);
    w.read_len.push_back(m);
    w.win_off.push_back(wo);
    w.win_len.push_back(n);
    w.mode.push_back((uint8_t)(rng() & 1));
    w.reads.resize(pos + m, 0);
    for (int i = 0; i < m; ++i) {
      // half copied from the window with an error or two, half random
      uint8_t c = (k & 1) && i < n ? w.ref[wo + i] : (uint8_t)(rng() & 3);
      if (rng() % 17 == 0) c = (uint8_t)((c + 1) & 3);
      w.reads[pos + i] = c;
    }
    pos += m;
  }
  w.reads.resize(pos + 32, 0);
  w.words.assign((w.reads.size() + 15) / 16, 0);
  for (size_t i = 0; i < w.reads.size(); ++i) w.words[i / 16] |= (uint32_t)w.reads[i] << (2 * (i % 16));
  return w;
}

// The oracle on reads [first, first + count) alone: 7 arrays at stride count
// and kCap CIGAR words per read.
static void oracle_outputs(const World& w, int64_t first, int64_t count, std::vector<int32_t>* out,
                           std::vector<uint32_t>* cig) {
  const int64_t n = count;
  out->assign((size_t)(7 * n), 0);
  cig->assign((size_t)(n * kCap), 0);
  std::vector<int64_t> ro(n), wo(n);
  for (int64_t p = 0; p < n; ++p) {
    ro[(size_t)p] = (int64_t)w.read_off[(size_t)(first + p)];
    wo[(size_t)p] = (int64_t)w.win_off[(size_t)(first + p)];
  }
  int32_t* o = out->data();
  oracle_align_batch(w.ref.data(), (int64_t)w.ref.size(), wo.data(), w.win_len.data() + first, w.reads.data(),
                     (int64_t)w.reads.size(), ro.data(), w.read_len.data() + first, w.mode.data() + first, 0, n, 1, -4,
                     6, 1, 1, kCap, o, o + 3 * n, o + n, o + 4 * n, o + 2 * n, cig->data(), o + 5 * n,
                     (uint32_t*)(o + 6 * n), 1);
}

// A slot that runs its batch with the oracle, after a random delay; it
// records what it was given.
class HostSlot : public Backend {
 public:
  HostSlot(const World* w, uint32_t seed, int max_delay_us, std::atomic<int>* in_flight, std::atomic<int>* peak,
           std::mutex* log_mu, std::vector<std::vector<uint64_t>>* log, uint64_t fail_id)
      : w_(w), rng_(seed), max_delay_us_(max_delay_us), in_flight_(in_flight), peak_(peak), log_mu_(log_mu),
        log_(log), fail_id_(fail_id) {}

  bool start(const Batch& b, std::string* err) override {
    const int now = ++*in_flight_;
    int p = peak_->load();
    while (now > p && !peak_->compare_exchange_weak(p, now)) {
    }
    std::vector<uint64_t> ids;
    for (auto& r : b.reqs) ids.push_back(r->id);
    {
      std::lock_guard<std::mutex> g(*log_mu_);
      log_->push_back(ids);
    }
    for (auto& r : b.reqs)
      if (r->id == fail_id_) {
        --*in_flight_;
        *err = "injected failure";
        return false;
      }
    // unpack the batch as a GPU slot stages it: reads back to back
    const int64_t n = b.n_pairs;
    std::vector<uint8_t> codes;
    std::vector<int64_t> ro, wo;
    std::vector<int32_t> rl, wl;
    std::vector<uint8_t> md;
    for (auto& r : b.reqs) {
      const int64_t base = (int64_t)codes.size();
      for (uint32_t word : r->reads)
        for (int t = 0; t < 16; ++t) codes.push_back((uint8_t)((word >> (2 * t)) & 3u));
      for (int64_t q = 0; q < r->n; ++q) {
        ro.push_back(base + (int64_t)r->read_off[(size_t)q]);
        wo.push_back((int64_t)r->win_off[(size_t)q]);
        rl.push_back(r->read_len[(size_t)q]);
        wl.push_back(r->win_len[(size_t)q]);
        md.push_back(r->mode.empty() ? 0 : r->mode[(size_t)q]);
      }
    }
    codes.resize(codes.size() + 16, 0);
    out_.assign((size_t)(7 * n), 0);
    cig_.assign((size_t)(n * kCap), 0);
    int32_t* o = out_.data();
    if (n)
      oracle_align_batch(w_->ref.data(), (int64_t)w_->ref.size(), wo.data(), wl.data(), codes.data(),
                         (int64_t)codes.size(), ro.data(), rl.data(), md.data(), 0, n, 1, -4, 6, 1, 1, kCap, o,
                         o + 3 * n, o + n, o + 4 * n, o + 2 * n, cig_.data(), o + 5 * n, (uint32_t*)(o + 6 * n), 1);
    delay();
    return true;
  }
  bool finish(std::string*) override {
    delay();
    --*in_flight_;
    return true;
  }
  const int32_t* outputs() const override { return out_.data(); }
  const uint32_t* cigars() const override { return cig_.data(); }
  // a plan is taken only while no slot runs a batch
  bool load_plan(const char* path, std::string* err) override {
    if (in_flight_->load() != 0) {
      *err = "plan loaded during a batch";
      return false;
    }
    plans_.push_back(path);
    return true;
  }
  std::vector<std::string> plans_;

 private:
  void delay() {
    if (max_delay_us_ > 0)
      std::this_thread::sleep_for(std::chrono::microseconds(std::uniform_int_distribution<int>(0, max_delay_us_)(rng_)));
  }
  const World* w_;
  std::mt19937 rng_;
  int max_delay_us_;
  std::atomic<int>* in_flight_;
  std::atomic<int>* peak_;
  std::mutex* log_mu_;
  std::vector<std::vector<uint64_t>>* log_;
  uint64_t fail_id_;
  std::vector<int32_t> out_;
  std::vector<uint32_t> cig_;
};

struct Rig {
  std::atomic<int> in_flight{0}, peak{0};
  std::mutex log_mu;
  std::vector<std::vector<uint64_t>> log;
  std::unique_ptr<Core> core;
  Rig(const World& w, int slots, Limits lim, int max_delay_us, uint64_t fail_id = ~0ull) {
    std::vector<std::unique_ptr<Backend>> b;
    for (int i = 0; i < slots; ++i)
      b.push_back(std::make_unique<HostSlot>(&w, 100u + (uint32_t)i, max_delay_us, &in_flight, &peak, &log_mu, &log,
                                             fail_id));
    core = std::make_unique<Core>(lim, std::move(b));
  }
};

struct Req {
  int64_t first, count;
};

static std::vector<Req> make_requests(const World& w, int n_req, uint32_t seed, int max_size) {
  std::mt19937 rng(seed);
  std::vector<Req> out;
  for (int r = 0; r < n_req; ++r) {
    const int64_t c = 1 + (int64_t)(rng() % (uint32_t)max_size);
    const int64_t f = (int64_t)(rng() % (uint32_t)(w.read_len.size() - (size_t)c));
    out.push_back({f, c});
  }
  return out;
}

static void submit_all(Core& core, const World& w, const std::vector<Req>& reqs, uint64_t id0) {
  for (size_t r = 0; r < reqs.size(); ++r) {
    std::string err;
    const auto& q = reqs[r];
    const mica_status_t st = core.submit(id0 + r, w.words.data(), w.read_off.data() + q.first,
                                         w.read_len.data() + q.first, w.win_off.data() + q.first,
                                         w.win_len.data() + q.first, w.mode.data() + q.first, q.count, -1.0, &err);
    CHECK(st == MICA_OK, "submit %zu: %s", r, err.c_str());
  }
}

// Wait for ids [id0, id0 + n), fetch each and compare with the oracle alone;
// the request with id failed_id must instead report MICA_ST_INTERNAL for
// every read.  (With `a` and `b`: the ids of two submitting threads, 1000..
// and 5000..; `reqs` then maps id - id0 with padding between the two
// ranges.)  A poll hands out every finished id, so all the ids a case waits
// for are collected in one call.
static void collect_and_check(Core& core, const World& w, const std::vector<Req>& reqs, uint64_t id0,
                              const char* what, uint64_t failed_id = ~0ull, const std::vector<Req>* a = nullptr,
                              const std::vector<Req>* b = nullptr) {
  std::set<uint64_t> left;
  if (a && b) {
    for (size_t r = 0; r < a->size(); ++r) left.insert(1000 + r);
    for (size_t r = 0; r < b->size(); ++r) left.insert(5000 + r);
  } else {
    for (size_t r = 0; r < reqs.size(); ++r) left.insert(id0 + r);
  }
  std::set<uint64_t> seen;
  const auto t0 = std::chrono::steady_clock::now();
  while (!left.empty()) {
    uint64_t ids[256];
    const int64_t k = core.poll(ids, 256);
    for (int64_t i = 0; i < k; ++i) {
      CHECK(!seen.count(ids[i]), "%s: id %llu polled twice", what, (unsigned long long)ids[i]);
      seen.insert(ids[i]);
      if (!left.count(ids[i])) continue;
      left.erase(ids[i]);
      const Req& q = reqs[(size_t)(ids[i] - id0)];
      const int64_t n = q.count;
      std::vector<int32_t> got((size_t)(7 * n)), want;
      std::vector<uint32_t> gcig((size_t)(n * kCap), 0xDEADBEEFu), wcig;
      std::string err;
      mica_status_t st = core.fetch(ids[i], got.data(), got.data() + 3 * n, got.data() + n, got.data() + 4 * n,
                                    got.data() + 2 * n, gcig.data(), kCap, got.data() + 5 * n,
                                    (uint32_t*)(got.data() + 6 * n), &err);
      CHECK(st == MICA_OK, "%s: fetch %llu: %s", what, (unsigned long long)ids[i], err.c_str());
      st = core.fetch(ids[i], nullptr, nullptr, nullptr, nullptr, nullptr, nullptr, 0, nullptr, nullptr, &err);
      CHECK(st == MICA_ERR_INVALID_ARG, "%s: a fetched request is forgotten", what);
      if (ids[i] == failed_id) {
        for (int64_t p = 0; p < n; ++p)
          CHECK((uint32_t)got[(size_t)(6 * n + p)] == (uint32_t)MICA_ST_INTERNAL, "%s: status of a failed batch",
                what);
        continue;
      }
      oracle_outputs(w, q.first, q.count, &want, &wcig);
      bool same = true;
      for (size_t x = 0; x < got.size(); ++x) same &= got[x] == want[x];
      for (int64_t p = 0; p < n && same; ++p) {
        const int32_t nc = want[(size_t)(5 * n + p)];
        const int32_t k = std::min<int32_t>(nc < 0 ? -nc : nc, kCap);
        for (int32_t y = 0; y < k; ++y) same &= gcig[(size_t)(p * kCap + y)] == wcig[(size_t)(p * kCap + y)];
      }
      CHECK(same, "%s: request %llu differs from the oracle on it alone", what, (unsigned long long)ids[i]);
    }
    if (std::chrono::steady_clock::now() - t0 > std::chrono::seconds(60)) {
      CHECK(false, "%s: %zu requests never finished", what, left.size());
      break;
    }
    std::this_thread::sleep_for(std::chrono::microseconds(200));
  }
}

int main() {
  const World w = make_world(6000, 7);
  Limits lim;
  lim.slot_pairs = 300;
  lim.slot_words = 900;
  lim.cigar_cap = kCap;

  // 1. continuous batching over 3 slots, two submitting threads, injected
  //    delays: exact results per request, limits, queue order, slot reuse
  {
    Rig rig(w, 3, lim, 2000);
    const auto reqs = make_requests(w, 400, 11, 120);
    std::vector<Req> a(reqs.begin(), reqs.begin() + 200), b(reqs.begin() + 200, reqs.end());
    std::thread t1([&] { submit_all(*rig.core, w, a, 1000); });
    std::thread t2([&] { submit_all(*rig.core, w, b, 5000); });
    t1.join();
    t2.join();
    // one collector: ids 1000.. and 5000.. map into one request list
    std::vector<Req> pad(4000 - a.size(), Req{0, 1});
    std::vector<Req> joined(a);
    joined.insert(joined.end(), pad.begin(), pad.end());
    joined.insert(joined.end(), b.begin(), b.end());
    collect_and_check(*rig.core, w, joined, 1000, "batching (two threads)", ~0ull, &a, &b);
    const auto runs = rig.core->batches_run();
    int64_t total = 0;
    for (int64_t x : runs) {
      CHECK(x >= 2, "every slot is reused (ran %lld batches)", (long long)x);
      total += x;
    }
    std::lock_guard<std::mutex> g(rig.log_mu);
    CHECK((int64_t)rig.log.size() == total, "batches logged %zu vs run %lld", rig.log.size(), (long long)total);
    CHECK(rig.peak.load() >= 2, "slots overlap (peak %d in flight)", rig.peak.load());
    size_t multi = 0;
    for (const auto& ids : rig.log) {
      int64_t pairs = 0, words = 0;
      for (uint64_t id : ids) {
        const Req& q = id >= 5000 ? b[(size_t)(id - 5000)] : a[(size_t)(id - 1000)];
        pairs += q.count;
        const uint64_t lo = w.read_off[(size_t)q.first] / 16;
        const uint64_t hi = (w.read_off[(size_t)(q.first + q.count - 1)] + w.read_len[(size_t)(q.first + q.count - 1)] + 15) / 16;
        words += (int64_t)(hi - lo);
      }
      CHECK(pairs <= lim.slot_pairs && words <= lim.slot_words, "batch over the slot limits (%lld pairs)",
            (long long)pairs);
      multi += ids.size() > 1;
      // requests of one submitting thread keep their order inside a batch
      uint64_t last_a = 0, last_b = 0;
      for (uint64_t id : ids) {
        uint64_t& last = id >= 5000 ? last_b : last_a;
        CHECK(id > last, "batch takes requests in queue order");
        last = id;
      }
    }
    CHECK(multi > 0, "some batches hold several requests");
    double p50 = 0, p99 = 0, gc = 0;
    std::string err;
    CHECK(rig.core->stats(&p50, &p99, &gc, &err) == MICA_OK && p50 > 0 && p99 >= p50 && gc > 0, "statistics");
    // argument errors
    CHECK(rig.core->submit(1000000, w.words.data(), w.read_off.data(), w.read_len.data(), w.win_off.data(),
                           w.win_len.data(), nullptr, lim.slot_pairs + 1, -1, &err) == MICA_ERR_LIMIT,
          "request over one batch");
    CHECK(rig.core->fetch(424242, nullptr, nullptr, nullptr, nullptr, nullptr, nullptr, 0, nullptr, nullptr, &err) ==
              MICA_ERR_INVALID_ARG,
          "unknown id");
    std::vector<uint8_t> bad_mode(1, 2);
    CHECK(rig.core->submit(1000001, w.words.data(), w.read_off.data(), w.read_len.data(), w.win_off.data(),
                           w.win_len.data(), bad_mode.data(), 1, -1, &err) == MICA_ERR_INVALID_ARG,
          "mode 2 refused by the server");
  }
  // 2. a request id in use is refused until fetched; FIFO mode runs one
  //    request per batch with one slot
  {
    Limits fl = lim;
    fl.fifo = true;
    Rig rig(w, 1, fl, 500);
    const auto reqs = make_requests(w, 60, 12, 50);
    submit_all(*rig.core, w, reqs, 7);
    std::string err;
    CHECK(rig.core->submit(7, w.words.data(), w.read_off.data(), w.read_len.data(), w.win_off.data(),
                           w.win_len.data(), nullptr, 1, -1, &err) == MICA_ERR_INVALID_ARG,
          "duplicate id refused");
    collect_and_check(*rig.core, w, reqs, 7, "fifo");
    std::lock_guard<std::mutex> g(rig.log_mu);
    for (const auto& ids : rig.log) CHECK(ids.size() == 1, "fifo batch of %zu requests", ids.size());
    for (size_t k = 1; k < rig.log.size(); ++k) CHECK(rig.log[k][0] > rig.log[k - 1][0], "fifo order");
    CHECK(rig.peak.load() == 1, "one slot never overlaps itself");
  }
  // 3. a failing batch: its requests finish with MICA_ST_INTERNAL, the
  //    others are exact, statistics report the error
  {
    Limits fl = lim;
    fl.fifo = true;
    Rig rig(w, 2, fl, 200, 3);
    const auto reqs = make_requests(w, 8, 13, 40);
    submit_all(*rig.core, w, reqs, 0);
    std::vector<Req> tail(reqs.begin() + 3, reqs.end());  // request 3 is in the failing batch
    collect_and_check(*rig.core, w, tail, 3, "failed batch and after", 3);
    double p50;
    std::string err;
    CHECK(rig.core->stats(&p50, nullptr, nullptr, &err) == MICA_ERR_HIP && err == "injected failure",
          "the error is reported (%s)", err.c_str());
  }
  // 4. replay: a schedule over 60 ms is submitted on time; latency counts
  //    from the scheduled arrival
  {
    Rig rig(w, 3, lim, 300);
    const auto reqs = make_requests(w, 200, 14, 60);
    std::vector<int64_t> first, count;
    std::vector<double> arr;
    const double t0 = rig.core->now() + 0.01;
    for (size_t r = 0; r < reqs.size(); ++r) {
      first.push_back(reqs[r].first);
      count.push_back(reqs[r].count);
      arr.push_back(t0 + 0.0003 * (double)r);
    }
    std::string err;
    CHECK(rig.core->replay(w.words.data(), w.read_off.data(), w.read_len.data(), w.win_off.data(), w.win_len.data(),
                           w.mode.data(), first.data(), count.data(), arr.data(), (int64_t)reqs.size(), 20000,
                           &err) == MICA_OK,
          "replay starts");
    CHECK(rig.core->replay(w.words.data(), w.read_off.data(), w.read_len.data(), w.win_off.data(), w.win_len.data(),
                           w.mode.data(), first.data(), count.data(), arr.data(), 1, 90000, &err) == MICA_ERR_BUSY,
          "one replay at a time");
    double lag = -1;
    CHECK(rig.core->replay_wait(&lag, &err) == MICA_OK && lag >= 0 && lag < 0.05, "replay lag %.4f s", lag);
    collect_and_check(*rig.core, w, reqs, 20000, "replayed");
  }
  // 5. a plan reaches every slot while none runs a batch, with submissions
  //    from another thread going on; every request still exact
  {
    Rig rig(w, 3, lim, 1500);
    const auto reqs = make_requests(w, 240, 16, 120);
    std::vector<Req> a(reqs.begin(), reqs.begin() + 120), b(reqs.begin() + 120, reqs.end());
    std::thread t1([&] { submit_all(*rig.core, w, a, 70000); });
    std::string err;
    for (int k = 0; k < 3; ++k) {
      std::this_thread::sleep_for(std::chrono::milliseconds(5));
      CHECK(rig.core->load_plan("plan.json", &err) == MICA_OK, "plan %d loads: %s", k, err.c_str());
    }
    t1.join();
    CHECK(rig.core->load_plan(nullptr, &err) == MICA_ERR_INVALID_ARG, "NULL plan path refused");
    // one id range for both sets, collected together (a poll hands out
    // every finished id, whichever set it belongs to)
    submit_all(*rig.core, w, b, 70000 + a.size());
    collect_and_check(*rig.core, w, reqs, 70000, "around and after plan loads");
    CHECK(rig.core->plans_loaded() == 3, "three plans loaded (%lld)", (long long)rig.core->plans_loaded());
    CHECK(rig.log.size() > 0, "batches ran");
  }
  // 6. stopping finishes what is queued
  {
    Rig rig(w, 2, lim, 1000);
    const auto reqs = make_requests(w, 50, 15, 100);
    submit_all(*rig.core, w, reqs, 0);
    rig.core->stop();
    uint64_t ids[64];
    int64_t n_done = 0, k;
    while ((k = rig.core->poll(ids, 64)) > 0) n_done += k;
    CHECK(n_done == (int64_t)reqs.size(), "stop finished %lld of %zu", (long long)n_done, reqs.size());
  }
  if (g_failures) {
    std::fprintf(stderr, "%d checks failed\n", g_failures);
    return 1;
  }
  std::printf("serving test double: all checks passed\n");
  return 0;
}
