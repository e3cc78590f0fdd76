// FM index of the reference for the few-mismatch search phase: suffix array
// by induced sorting (SA-IS), BWT, occurrence blocks, upload to the device.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <cstring>
#include <new>
#include <string>
#include <vector>

#include "ctx.h"
#include "fm_common.h"
#include "mica_fm.h"

namespace {

constexpr uint32_t kEmpty = 0xFFFFFFFFu;

// Suffix array of T[0, n) over symbols 0..K-1 where T[n-1] = 0 is the unique
// smallest symbol (the sentinel), by induced sorting (Nong, Zhang & Chan,
// "Two efficient algorithms for linear time suffix array construction"):
// classify suffixes as S or L, sort the LMS substrings by one round of
// induction, name them, solve the reduced string (recursively when names
// repeat), then induce the full order from the sorted LMS suffixes.
template <class Sym>
void sais(const Sym* T, uint32_t* SA, uint32_t n, uint32_t K) {
  if (n == 1) {
    SA[0] = 0;
    return;
  }
  std::vector<uint8_t> stype(n);  // 1: S-type suffix
  stype[n - 1] = 1;
  for (int64_t i = (int64_t)n - 2; i >= 0; --i)
    stype[i] = (T[i] < T[i + 1] || (T[i] == T[i + 1] && stype[i + 1])) ? 1 : 0;
  auto is_lms = [&](uint32_t i) { return i > 0 && i != kEmpty && stype[i] && !stype[i - 1]; };
  std::vector<uint32_t> cnt(K, 0), bkt(K);
  for (uint32_t i = 0; i < n; ++i) cnt[T[i]]++;
  auto bucket_ends = [&]() {
    uint32_t s = 0;
    for (uint32_t c = 0; c < K; ++c) {
      s += cnt[c];
      bkt[c] = s;
    }
  };
  auto bucket_starts = [&]() {
    uint32_t s = 0;
    for (uint32_t c = 0; c < K; ++c) {
      bkt[c] = s;
      s += cnt[c];
    }
  };
  // L-type suffixes left to right from bucket starts, then S-type right to
  // left from bucket ends
  auto induce = [&]() {
    bucket_starts();
    for (uint32_t i = 0; i < n; ++i) {
      const uint32_t s = SA[i];
      if (s != kEmpty && s > 0 && !stype[s - 1]) SA[bkt[T[s - 1]]++] = s - 1;
    }
    bucket_ends();
    for (int64_t i = (int64_t)n - 1; i >= 0; --i) {
      const uint32_t s = SA[i];
      if (s != kEmpty && s > 0 && stype[s - 1]) SA[--bkt[T[s - 1]]] = s - 1;
    }
  };

  // 1. LMS suffixes at the ends of their buckets, then one induction sorts
  //    the LMS substrings
  std::fill(SA, SA + n, kEmpty);
  bucket_ends();
  for (uint32_t i = 1; i < n; ++i)
    if (is_lms(i)) SA[--bkt[T[i]]] = i;
  induce();

  // 2. sorted LMS substrings to the front; name them (equal substrings share
  //    a name), names stored at SA[n1 + pos / 2] (LMS positions are >= 2 apart)
  uint32_t n1 = 0;
  for (uint32_t i = 0; i < n; ++i)
    if (is_lms(SA[i])) SA[n1++] = SA[i];
  std::fill(SA + n1, SA + n, kEmpty);
  uint32_t names = 0, prev = kEmpty;
  for (uint32_t i = 0; i < n1; ++i) {
    const uint32_t pos = SA[i];
    bool diff = prev == kEmpty;
    for (uint32_t d = 0; !diff; ++d) {
      if (T[pos + d] != T[prev + d] || stype[pos + d] != stype[prev + d]) {
        diff = true;
      } else if (d > 0 && is_lms(pos + d)) {
        break;  // both substrings end here, equal (their types agree)
      }
    }
    if (diff) {
      ++names;
      prev = pos;
    }
    SA[n1 + pos / 2] = names - 1;
  }
  // names in text order at the end of SA: the reduced string S1
  {
    uint32_t j = n - 1;
    for (int64_t i = (int64_t)n - 1; i >= (int64_t)n1; --i)
      if (SA[i] != kEmpty) SA[j--] = SA[i];
  }
  uint32_t* S1 = SA + n - n1;
  uint32_t* SA1 = SA;

  // 3. order of the LMS suffixes
  if (names < n1) {
    sais<uint32_t>(S1, SA1, n1, names);
  } else {
    for (uint32_t i = 0; i < n1; ++i) SA1[S1[i]] = i;
  }

  // 4. sorted LMS suffixes at their bucket ends, induce the rest
  {
    uint32_t j = 0;
    for (uint32_t i = 1; i < n; ++i)
      if (is_lms(i)) S1[j++] = i;  // LMS positions in text order
  }
  for (uint32_t i = 0; i < n1; ++i) SA1[i] = S1[SA1[i]];
  std::fill(SA + n1, SA + n, kEmpty);
  bucket_ends();
  for (int64_t i = (int64_t)n1 - 1; i >= 0; --i) {
    const uint32_t p = SA[i];
    SA[i] = kEmpty;
    SA[--bkt[T[p]]] = p;
  }
  induce();
}

// suffix array of codes[0, n) + sentinel into sa[0, n] (codes validated)
void suffix_array(const uint8_t* codes, uint64_t n, uint32_t* sa) {
  std::vector<uint8_t> T(n + 1);
  for (uint64_t i = 0; i < n; ++i) T[i] = (uint8_t)(codes[i] + 1);
  T[n] = 0;
  sais<uint8_t>(T.data(), sa, (uint32_t)(n + 1), 5);
}

}  // namespace

struct mica_fm {
  int device = 0;
  mica::FmIndex ix{};
  void* d_occ = nullptr;
  void* d_sa = nullptr;
  void* d_ref = nullptr;
  uint64_t bytes = 0;
  double build_s = 0;
};

extern "C" mica_status_t mica_fm_suffix_array(const uint8_t* codes, uint64_t n, uint32_t* sa) {
  if (!sa || (n > 0 && !codes)) return mica::fail(MICA_ERR_INVALID_ARG, "NULL codes or sa");
  if (n > MICA_FM_MAX_REF_LEN) return mica::fail(MICA_ERR_LIMIT, "text longer than MICA_FM_MAX_REF_LEN");
  for (uint64_t i = 0; i < n; ++i)
    if (codes[i] > 3) return mica::fail(MICA_ERR_INVALID_ARG, "base code above 3");
  try {
    suffix_array(codes, n, sa);
  } catch (const std::bad_alloc&) {
    return mica::fail(MICA_ERR_OUT_OF_MEMORY, "host memory for the suffix array construction");
  }
  return MICA_OK;
}

namespace {

mica_status_t release(mica_fm* f) {
  if (f->d_occ) (void)hipFree(f->d_occ);
  if (f->d_sa) (void)hipFree(f->d_sa);
  if (f->d_ref) (void)hipFree(f->d_ref);
  delete f;
  return MICA_OK;
}

mica_status_t build(mica_fm* f, const uint32_t* host_ref2b, uint64_t n) {
  using namespace mica;
  // codes, suffix array, BWT
  std::vector<uint8_t> codes(n);
  for (uint64_t i = 0; i < n; ++i) codes[i] = (uint8_t)((host_ref2b[i >> 4] >> (2 * (i & 15))) & 3u);
  std::vector<uint32_t> sa(n + 1);
  suffix_array(codes.data(), n, sa.data());
  const uint64_t rows = n + 1;
  const uint64_t nblk = rows / kFmBlockSyms + 1;
  std::vector<uint32_t> occ(nblk * kFmBlockWords, 0u);
  uint32_t run[4] = {0, 0, 0, 0};
  uint32_t dollar = 0;
  for (uint64_t i = 0; i < rows; ++i) {
    const uint64_t b = i / kFmBlockSyms, o = i % kFmBlockSyms;
    uint32_t* blk = occ.data() + b * kFmBlockWords;
    if (o == 0)
      for (int c = 0; c < 4; ++c) blk[c] = run[c];
    uint32_t sym = 0;  // the sentinel row stores symbol 0 and is not counted
    if (sa[i] == 0) {
      dollar = (uint32_t)i;
    } else {
      sym = codes[sa[i] - 1];
      run[sym]++;
    }
    blk[4 + o / 16] |= sym << (2 * (o % 16));
  }
  // queries reach row index n + 1: when it starts a block of its own, that
  // block holds the totals (and no symbols)
  for (uint64_t b = (rows - 1) / kFmBlockSyms + 1; b < nblk; ++b)
    for (int c = 0; c < 4; ++c) occ[b * kFmBlockWords + c] = run[c];
  f->ix.n = n;
  f->ix.dollar = dollar;
  f->ix.device = f->device;
  uint32_t acc = 1;  // row 0 is the sentinel suffix
  for (int c = 0; c < 4; ++c) {
    f->ix.C[c] = acc;
    acc += run[c];
  }
  const uint64_t ref_words = (n + 15) / 16 + 2;  // padded for two-word reads at the end
  std::vector<uint32_t> refw(ref_words, 0u);
  std::memcpy(refw.data(), host_ref2b, ((n + 15) / 16) * 4);
  if (n % 16) refw[n / 16] &= (1u << (2 * (n % 16))) - 1;
  HIP_TRY(hipSetDevice(f->device));
  HIP_TRY(hipMalloc(&f->d_occ, occ.size() * 4));
  HIP_TRY(hipMalloc(&f->d_sa, rows * 4));
  HIP_TRY(hipMalloc(&f->d_ref, ref_words * 4));
  HIP_TRY(hipMemcpy(f->d_occ, occ.data(), occ.size() * 4, hipMemcpyHostToDevice));
  HIP_TRY(hipMemcpy(f->d_sa, sa.data(), rows * 4, hipMemcpyHostToDevice));
  HIP_TRY(hipMemcpy(f->d_ref, refw.data(), ref_words * 4, hipMemcpyHostToDevice));
  f->ix.occ = (const uint32_t*)f->d_occ;
  f->ix.sa = (const uint32_t*)f->d_sa;
  f->ix.ref2b = (const uint32_t*)f->d_ref;
  f->ix.ref_words = ref_words;
  f->bytes = occ.size() * 4 + rows * 4 + ref_words * 4;
  return MICA_OK;
}

}  // namespace

namespace mica {
const FmIndex* fm_index_of(const mica_fm* f) { return &f->ix; }
}  // namespace mica

extern "C" mica_status_t mica_fm_create(int hip_device, const uint32_t* host_ref2b, uint64_t ref_len,
                                        mica_fm_t* out) {
  if (!out) return mica::fail(MICA_ERR_INVALID_ARG, "NULL out");
  *out = nullptr;
  if (!host_ref2b || ref_len == 0) return mica::fail(MICA_ERR_INVALID_ARG, "empty reference");
  if (ref_len > MICA_FM_MAX_REF_LEN) return mica::fail(MICA_ERR_LIMIT, "reference longer than MICA_FM_MAX_REF_LEN");
  int ndev = 0;
  if (hipGetDeviceCount(&ndev) != hipSuccess || hip_device < 0 || hip_device >= ndev)
    return mica::fail(MICA_ERR_HIP, "no such HIP device");
  mica_fm* f = new (std::nothrow) mica_fm();
  if (!f) return mica::fail(MICA_ERR_OUT_OF_MEMORY, "host memory");
  f->device = hip_device;
  const auto t0 = std::chrono::steady_clock::now();
  mica_status_t st;
  try {
    st = build(f, host_ref2b, ref_len);
  } catch (const std::bad_alloc&) {
    st = mica::fail(MICA_ERR_OUT_OF_MEMORY, "host memory for the index build");
  }
  if (st != MICA_OK) {
    release(f);
    return st;
  }
  f->build_s = std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
  *out = f;
  return MICA_OK;
}

extern "C" mica_status_t mica_fm_destroy(mica_fm_t f) {
  if (!f) return MICA_OK;
  (void)hipSetDevice(f->device);
  (void)hipDeviceSynchronize();
  return release(f);
}

extern "C" mica_status_t mica_fm_info(mica_fm_t f, uint64_t* device_bytes, double* build_seconds) {
  if (!f) return mica::fail(MICA_ERR_INVALID_ARG, "NULL index");
  if (device_bytes) *device_bytes = f->bytes;
  if (build_seconds) *build_seconds = f->build_s;
  return MICA_OK;
}
