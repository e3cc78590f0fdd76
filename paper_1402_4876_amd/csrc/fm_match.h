// Base comparisons of the few-mismatch search (Methods, architecture &
// parallelism: a read placed with few mismatches): 2-bit words of 16 bases,
// a read stretch against a reference stretch 16 bases at a time.
//
// Plain integer code, used by the search kernel (fm_search.hip) and built as
// host C++ by the sanitizer checks of the CPU tests (which define the
// __host__ / __device__ / __forceinline__ keywords away).
#pragma once
#include <stdint.h>

namespace mica {
namespace fm {

// base p of a 2-bit word array
__host__ __device__ __forceinline__ uint32_t base_at(const uint32_t* w, uint64_t p) {
  return (w[p >> 4] >> (2 * (uint32_t)(p & 15))) & 3u;
}

// 16 bases from base position p (zeros past the last of the nwords words):
// the low 32 bits of the 64-bit pair (w[i + 1], w[i]) shifted right by 2 (p mod 16)
__host__ __device__ __forceinline__ uint32_t bases16(const uint32_t* w, uint64_t p, uint64_t nwords) {
  const uint64_t i = p >> 4;
  const uint32_t s = 2 * (uint32_t)(p & 15);
  const uint32_t lo = i < nwords ? w[i] : 0u;
  if (s == 0) return lo;
  const uint32_t hi = i + 1 < nwords ? w[i + 1] : 0u;
  return (uint32_t)((((uint64_t)hi << 32) | lo) >> s);
}

// bit 2t set where symbol t of the two 16-base words differs
__host__ __device__ __forceinline__ uint32_t diff_mask(uint32_t a, uint32_t b) {
  const uint32_t x = a ^ b;
  return (x | (x >> 1)) & 0x55555555u;
}

// the symbols t of a 16-base chunk with t < rem (1 <= rem; rem >= 16 keeps all)
__host__ __device__ __forceinline__ uint32_t low_symbols(uint32_t m, int rem) {
  return rem >= 16 ? m : m & ((1u << (2 * rem)) - 1u);
}

// A read stretch and a reference stretch: 2-bit words and their counts.
struct Stretch {
  const uint32_t* reads;
  uint64_t read_words;
  const uint32_t* ref;
  uint64_t ref_words;
};

// difference mask of the 16 read bases from ro + t and the reference bases
// from p + t, the symbols at or past len cleared
__host__ __device__ __forceinline__ uint32_t chunk_diff(const Stretch& S, uint64_t ro, uint64_t p, int t, int len) {
  return low_symbols(diff_mask(bases16(S.reads, ro + t, S.read_words), bases16(S.ref, p + t, S.ref_words)),
                     len - t);
}

// mismatches between read bases [ro, ro + len) and reference bases
// [p, p + len); the count stops growing once it exceeds lim
__host__ __device__ __forceinline__ int mismatches(const Stretch& S, uint64_t ro, uint64_t p, int len, int lim) {
  int d = 0;
  for (int t = 0; t < len; t += 16) {
    d += __builtin_popcount(chunk_diff(S, ro, p, t, len));
    if (d > lim) break;
  }
  return d;
}

// read bases [ro, ro + len) equal reference bases [p, p + len)
__host__ __device__ __forceinline__ bool exact(const Stretch& S, uint64_t ro, uint64_t p, int len) {
  uint32_t acc = 0;
  for (int t = 0; t < len; t += 16) acc |= chunk_diff(S, ro, p, t, len);
  return acc == 0;
}

}  // namespace fm
}  // namespace mica
