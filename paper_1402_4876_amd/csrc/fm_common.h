// FM index layout shared by the index build (host) and the search kernel.
#pragma once
#include <cstdint>

struct mica_fm;

namespace mica {

// occurrence block: counts of A, C, G, T in the BWT before the block, then
// 192 BWT symbols as twelve words of 2-bit codes (64 bytes, one cache line)
constexpr int kFmBlockSyms = 192;
constexpr int kFmBlockWords = 16;

struct FmIndex {
  const uint32_t* occ;  // (n + 1) / 192 + 1 blocks
  const uint32_t* sa;   // n + 1 suffix starts; row 0 is the sentinel suffix
  const uint32_t* ref2b;  // reference, 2-bit words, two words of zero padding
  uint64_t n;           // reference length
  uint64_t ref_words;
  uint32_t C[4];        // first row of the suffixes starting with each base
  uint32_t dollar;      // BWT row holding the sentinel (stored as code 0, not counted)
  int device;           // HIP device holding the index
};

const FmIndex* fm_index_of(const mica_fm* f);

}  // namespace mica
