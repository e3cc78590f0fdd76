// Driver for the CPU oracle built with AddressSanitizer and
// UndefinedBehaviorSanitizer (tests/test_serve_double.py): every entry point
// on hand examples, empty and boundary lengths, pairs over the limits, reads
// and windows outside their buffers, several thread counts and random
// batches in all three modes; a few closed forms are checked on the way.
// Exit status 0 = no sanitizer report and every check passed.
#include <cstdint>
#include <cstdio>
#include <random>
#include <vector>

extern "C" {
int oracle_align_batch_ext(const uint8_t* ref, int64_t ref_len, const int64_t* win_off, const int32_t* win_len,
                           const uint8_t* reads, int64_t reads_len, const int64_t* read_off, const int32_t* read_len,
                           const uint8_t* mode, int32_t default_mode, const int32_t* h0, int32_t default_h0,
                           int32_t clip, int64_t n_pairs, int32_t match, int32_t mismatch, int32_t gap_open,
                           int32_t gap_extend, int32_t want_trace, int32_t cigar_cap, int32_t* score,
                           int32_t* read_start, int32_t* read_end, int32_t* ref_start, int32_t* ref_end,
                           uint32_t* cigar, int32_t* n_cigar, uint32_t* status, int32_t n_threads);
int oracle_kmm_search(const uint8_t* ref, int64_t ref_len, const uint8_t* reads, int64_t reads_len,
                      const int64_t* read_off, const int32_t* read_len, int64_t n_reads, int32_t k, int32_t max_occ,
                      int32_t* best_mm, int32_t* n_best, int32_t* n_hits, int64_t* pos, uint32_t* status,
                      int32_t n_threads);
}

static int failures = 0;
#define CHECK(c, msg)                                              \
  do {                                                             \
    if (!(c)) {                                                    \
      std::fprintf(stderr, "CHECK failed line %d: %s\n", __LINE__, msg); \
      ++failures;                                                  \
    }                                                              \
  } while (0)

struct Out {
  std::vector<int32_t> score, rs, re, fs, fe, nc;
  std::vector<uint32_t> cig, st;
  Out(size_t n, int cap) : score(n), rs(n), re(n), fs(n), fe(n), nc(n), cig(n * (size_t)(cap ? cap : 1)), st(n) {}
};

int main() {
  std::mt19937 rng(5);
  const int n_ref = 30000;
  std::vector<uint8_t> ref(n_ref);
  for (auto& c : ref) c = (uint8_t)(rng() & 3);
  // random batches in all modes, with traceback, several thread counts and capacities
  for (int round = 0; round < 4; ++round) {
    const int n = 300;
    std::vector<int64_t> wo(n), ro(n);
    std::vector<int32_t> wl(n), rl(n), h0(n);
    std::vector<uint8_t> md(n), reads;
    for (int p = 0; p < n; ++p) {
      rl[p] = (int)(rng() % 120);
      wl[p] = (int)(rng() % 200);
      wo[p] = (int64_t)(rng() % (uint32_t)(n_ref - 200));
      md[p] = (uint8_t)(rng() % 3);
      h0[p] = (int32_t)(rng() % 50);
      ro[p] = (int64_t)reads.size() + (int64_t)(rng() % 3);
      reads.resize((size_t)ro[p]);
      for (int i = 0; i < rl[p]; ++i)
        reads.push_back(i < wl[p] && (p & 1) ? ref[(size_t)(wo[p] + i)] : (uint8_t)(rng() & 3));
    }
    const int cap = round == 3 ? 0 : 1 + round * 20;
    Out o(n, cap);
    const int rc = oracle_align_batch_ext(ref.data(), n_ref, wo.data(), wl.data(), reads.data(), (int64_t)reads.size(),
                                          ro.data(), rl.data(), md.data(), 0, h0.data(), 0, 5, n, 1, -4, 6, 1, 1, cap,
                                          o.score.data(), o.rs.data(), o.re.data(), o.fs.data(), o.fe.data(),
                                          o.cig.data(), o.nc.data(), o.st.data(), 1 + round);
    CHECK(rc == 0, "random batch accepted");
    for (int p = 0; p < n; ++p) CHECK(md[p] != 1 || o.score[p] >= 0, "local scores are >= 0");
  }
  // identity, empty and boundary cases; out-of-range pairs set status bits
  {
    std::vector<uint8_t> q(ref.begin(), ref.begin() + 1024);
    std::vector<int64_t> wo = {0, 0, 0, 5, n_ref - 10, 0, 100};
    std::vector<int32_t> wl = {1024, 0, 5, 0, 20, 8192, 3000};
    std::vector<int64_t> ro = {0, 0, 0, 0, 0, 2000, 0};
    std::vector<int32_t> rl = {1024, 10, 0, 0, 5, 5, 1025};
    const int n = (int)wo.size();
    Out o(n, 64);
    const int rc = oracle_align_batch_ext(ref.data(), n_ref, wo.data(), wl.data(), q.data(), (int64_t)q.size(),
                                          ro.data(), rl.data(), nullptr, 0, nullptr, 0, 0, n, 1, -4, 6, 1, 1, 64,
                                          o.score.data(), o.rs.data(), o.re.data(), o.fs.data(), o.fe.data(),
                                          o.cig.data(), o.nc.data(), o.st.data(), 2);
    CHECK(rc == 0, "edge batch accepted");
    CHECK(o.score[0] == 1024, "identical 1024-base read scores m * a");
    CHECK(o.score[1] == -(6 + 10), "empty window: all insertions");
    CHECK(o.score[2] == 0 && o.st[2] == 0, "empty read");
    CHECK(o.st[4] != 0, "window past the reference end is flagged");
    CHECK(o.st[5] != 0, "read outside its buffer is flagged");
    CHECK(o.st[6] != 0, "read over 1024 bases is flagged");
  }
  // bad scoring is refused
  {
    int32_t s = 0, z = 0;
    uint32_t st = 0;
    int64_t zo = 0;
    int32_t zl = 0;
    CHECK(oracle_align_batch_ext(ref.data(), n_ref, &zo, &zl, ref.data(), 1, &zo, &zl, nullptr, 0, nullptr, 0, 0, 1,
                                 0, -4, 6, 1, 0, 0, &s, nullptr, &z, nullptr, &z, nullptr, nullptr, &st, 1) != 0,
          "match 0 refused");
  }
  // few-mismatch search: planted reads, random reads, reads at both ends, too short
  {
    const int n = 200;
    std::vector<int64_t> ro(n);
    std::vector<int32_t> rl(n);
    std::vector<uint8_t> reads;
    for (int r = 0; r < n; ++r) {
      rl[r] = r % 50 == 0 ? 2 : 30 + (int)(rng() % 90);
      const int64_t at = r % 7 == 0 ? 0 : (r % 11 == 0 ? n_ref - rl[r] : (int64_t)(rng() % (uint32_t)(n_ref - rl[r])));
      ro[r] = (int64_t)reads.size();
      for (int i = 0; i < rl[r]; ++i) reads.push_back(r % 3 ? ref[(size_t)(at + i)] : (uint8_t)(rng() & 3));
      if (rl[r] > 5 && r % 5 == 1) reads[(size_t)(ro[r] + rl[r] - 1)] ^= 1;
    }
    std::vector<int32_t> bm(n), nb(n), nh(n);
    std::vector<int64_t> pos(n);
    std::vector<uint32_t> st(n);
    for (int k = 0; k <= 2; ++k) {
      const int rc = oracle_kmm_search(ref.data(), n_ref, reads.data(), (int64_t)reads.size(), ro.data(), rl.data(), n, k,
                                       8, bm.data(), nb.data(), nh.data(), pos.data(), st.data(), 1 + k);
      CHECK(rc == 0, "search accepted");
      for (int r = 0; r < n; ++r)
        if (r % 3 && r % 5 != 1 && rl[r] >= 3 && st[r] == 0) CHECK(bm[r] == 0, "planted read found exactly");
    }
    CHECK(oracle_kmm_search(ref.data(), n_ref, reads.data(), 1, ro.data(), rl.data(), 0, 3, 8, bm.data(), nb.data(),
                            nh.data(), pos.data(), st.data(), 1) != 0,
          "k = 3 refused");
  }
  if (failures) {
    std::fprintf(stderr, "%d checks failed\n", failures);
    return 1;
  }
  std::printf("oracle under sanitizers: ok\n");
  return 0;
}
