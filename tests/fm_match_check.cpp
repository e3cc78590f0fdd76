// The few-mismatch search's base comparisons (paper_1402_4876_amd/csrc/fm_match.h)
// built as host code under AddressSanitizer + UndefinedBehaviorSanitizer
// (tests/test_serve_double.py): on random 2-bit words, at every alignment of
// read and reference offsets, for stretch lengths 1..1024 and placements
// that end on the last reference base, every helper is compared with a
// base-by-base count.  The word arrays are exactly as long as the data, so a
// read past them is an ASan report; the early-exit count used as an
// exactness test (mismatches with limit 0) is checked against exact().
// Exit status 0 = no sanitizer report and every check passed.
#include <cstdint>
#include <cstdio>
#include <random>
#include <vector>

#define __host__
#define __device__
#define __forceinline__ inline
#include "fm_match.h"

using mica::fm::Stretch;

static int failures = 0;
#define CHECK(c, ...)                                  \
  do {                                                 \
    if (!(c)) {                                        \
      if (failures < 20) std::fprintf(stderr, __VA_ARGS__); \
      ++failures;                                      \
    }                                                  \
  } while (0)

static std::vector<uint32_t> pack(const std::vector<uint8_t>& codes) {
  std::vector<uint32_t> w((codes.size() + 15) / 16, 0u);
  for (size_t i = 0; i < codes.size(); ++i) w[i / 16] |= (uint32_t)codes[i] << (2 * (i % 16));
  return w;
}

int main() {
  std::mt19937_64 rng(77);
  const int n_ref = 5000, n_reads = 3000;
  std::vector<uint8_t> ref(n_ref), reads(n_reads);
  for (auto& c : ref) c = (uint8_t)(rng() & 3);
  for (auto& c : reads) c = (uint8_t)(rng() & 3);
  // plant copies of reference stretches so that exact and near-exact
  // placements occur (with 0-3 substitutions)
  for (int k = 0; k < 40; ++k) {
    const int len = 1 + (int)(rng() % 300), ro = (int)(rng() % (n_reads - len)), p = (int)(rng() % (n_ref - len));
    for (int i = 0; i < len; ++i) reads[ro + i] = ref[p + i];
    for (int s = 0, ns = k % 4; s < ns; ++s) reads[ro + rng() % len] ^= 1;
  }
  const std::vector<uint32_t> rw = pack(reads), fw = pack(ref);
  const Stretch S{rw.data(), (uint64_t)rw.size(), fw.data(), (uint64_t)fw.size()};
  // base_at and bases16 (zeros past the data) at every position
  for (int p = 0; p < n_ref + 40; ++p) {
    if (p < n_ref) CHECK(mica::fm::base_at(fw.data(), p) == ref[p], "base_at %d\n", p);
    const uint32_t w = mica::fm::bases16(fw.data(), p, fw.size());
    for (int t = 0; t < 16; ++t) {
      const uint32_t want = p + t < n_ref ? ref[p + t] : 0u;
      CHECK(((w >> (2 * t)) & 3u) == want, "bases16 %d symbol %d\n", p, t);
    }
  }
  // stretches at random and at boundary offsets
  long checked = 0;
  for (int it = 0; it < 200000; ++it) {
    int len = it % 5 == 0 ? 1 + (int)(rng() % 1024) : 1 + (int)(rng() % 160);
    if (len > n_reads) len = n_reads;
    const uint64_t ro = rng() % (uint64_t)(n_reads - len + 1);
    uint64_t p = rng() % (uint64_t)(n_ref - len + 1);
    if (it % 7 == 0) p = (uint64_t)(n_ref - len);  // ends on the last base
    if (it % 11 == 0) p = ro % 16 + 16 * (rng() % ((n_ref - len) / 16 + 1));  // same alignment as the read
    if (p + len > (uint64_t)n_ref) p = (uint64_t)(n_ref - len);
    int naive = 0;
    for (int i = 0; i < len; ++i) naive += reads[ro + i] != ref[p + i];
    for (int lim : {0, 1, 2, 1 << 20}) {
      const int d = mica::fm::mismatches(S, ro, p, len, lim);
      if (naive <= lim) CHECK(d == naive, "mismatches ro %llu p %llu len %d lim %d: %d != %d\n",
                              (unsigned long long)ro, (unsigned long long)p, len, lim, d, naive);
      else CHECK(d > lim && d <= naive, "mismatches past the limit ro %llu p %llu len %d lim %d: %d (%d)\n",
                 (unsigned long long)ro, (unsigned long long)p, len, lim, d, naive);
    }
    const bool ex = mica::fm::exact(S, ro, p, len);
    CHECK(ex == (naive == 0), "exact ro %llu p %llu len %d: %d (%d mismatches)\n", (unsigned long long)ro,
          (unsigned long long)p, len, (int)ex, naive);
    CHECK((mica::fm::mismatches(S, ro, p, len, 0) == 0) == ex, "early-exit exactness ro %llu p %llu len %d\n",
          (unsigned long long)ro, (unsigned long long)p, len);
    // the last chunk's mask at every remainder
    for (int t = 0; t < len; t += 16) {
      const uint32_t m = mica::fm::chunk_diff(S, ro, p, t, len);
      for (int s = 0; s < 16; ++s) {
        const bool in = t + s < len;
        const bool want = in && reads[ro + t + s] != ref[p + t + s];
        CHECK((((m >> (2 * s)) & 1u) != 0) == want && ((m >> (2 * s + 1)) & 1u) == 0,
              "chunk_diff ro %llu p %llu len %d t %d s %d\n", (unsigned long long)ro, (unsigned long long)p, len, t, s);
      }
    }
    ++checked;
  }
  if (failures) {
    std::fprintf(stderr, "%d checks failed\n", failures);
    return 1;
  }
  std::printf("search base comparisons: %ld stretches ok\n", checked);
  return 0;
}
