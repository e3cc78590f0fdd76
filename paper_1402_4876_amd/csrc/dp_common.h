// Internal definitions shared by the device kernels and the host runtime of
// the DP-phase library.  Nothing here is part of the public C ABI.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace mica {

constexpr int kMaxM = 1024;  // longest read (rows)
constexpr int kMaxN = 8192;  // longest window (columns)
constexpr int kMaxH0 = 1 << 20;  // largest extension anchor score and clipping penalty

// Kernel classes: class c < 16 runs 16 lanes per pair with c+1 read rows per
// lane (reads up to 16*(c+1) bases); classes 16, 17 and 18 run a whole wave
// (64 lanes) with 16, 4 and 8 rows per lane (reads up to 1024, 256 and 512
// bases).  The default plan uses classes 0-16; 17 and 18 are alternatives a
// tuned plan may pick.
constexpr int kNumClasses = 19;
__host__ __device__ constexpr int class_lanes(int c) { return c < 16 ? 16 : 64; }
__host__ __device__ constexpr int class_rows(int c) { return c < 16 ? c + 1 : (c == 16 ? 16 : (c == 17 ? 4 : 8)); }
// class of (lanes, rows), or -1
__host__ __device__ constexpr int class_of(int lanes, int rows) {
  return lanes == 16 ? (rows >= 1 && rows <= 16 ? rows - 1 : -1)
                     : (lanes == 64 ? (rows == 16 ? 16 : (rows == 4 ? 17 : (rows == 8 ? 18 : -1))) : -1);
}

// Arithmetic kinds: packed 16-bit (two pairs per 32-bit register), packed
// 16-bit with a run-time saturation check, and 32-bit.
enum Kind : int { kK16 = 0, kK16Sat = 1, kK32 = 2 };
constexpr int kNumKinds = 3;
// alignment modes: 0 semi-global, 1 local, 2 seed extension with clipping
constexpr int kNumModes = 3;
constexpr int kNumBuckets = kNumKinds * kNumClasses * kNumModes;
__host__ __device__ constexpr int bucket_id(int kind, int cls, int mode) {
  return (kind * kNumClasses + cls) * kNumModes + mode;
}
__host__ __device__ constexpr int bucket_kind(int b) { return b / (kNumModes * kNumClasses); }
__host__ __device__ constexpr int bucket_class(int b) { return (b / kNumModes) % kNumClasses; }
__host__ __device__ constexpr int bucket_mode(int b) { return b % kNumModes; }
// Within a bucket pairs are ordered by read length, longest first, in
// kSubBins bins of the dummy-row count d0 (one bin per row for the 16-lane
// classes, 16 rows per bin for the 64-lane ones, the last bin open-ended).
// A work item then holds reads of nearly equal length and, since windows
// usually grow with the read, nearly equal windows: its step count (the
// longest window of its pairs) wastes less on its shorter pairs, and the
// longest items of a bucket are taken first.
constexpr int kSubBins = 16;
constexpr int kNumSubBuckets = kNumBuckets * kSubBins;
__host__ __device__ constexpr int sub_bin(int cls, int d0) {
  return (class_lanes(cls) == 16 ? d0 : d0 >> 4) < kSubBins - 1 ? (class_lanes(cls) == 16 ? d0 : d0 >> 4)
                                                                 : kSubBins - 1;
}
// pairs handled by one wave-sized work item
__host__ __device__ constexpr int pairs_per_item(int kind, int cls) {
  return (kind == kK32 ? 1 : 2) * (64 / class_lanes(cls));
}
// The class whose kernels may trace a pair of class `cls` back in full when
// its band is too wide.  For the 16-lane classes of 8 rows or more it is the
// 64-lane class of 4 rows (256 row slots): a fourth of the rows per lane, so
// one such item, which runs alone at the end of a small batch, takes about
// a third of the time, for more work per pair (the extra dummy rows).  The
// persistent side-list kernels always use it; a per-bucket side launch uses
// it while its list is short against the resident waves.  (The planner
// checks the 16-bit bounds with this class's dummy rows.)
__host__ __device__ constexpr int fallback_class(int cls) {
  return class_lanes(cls) == 16 && class_rows(cls) >= 8 ? 17 : cls;
}
static_assert(class_lanes(17) == 64 && class_rows(17) == 4, "the 256-row class of 64 lanes");

// The persistent kernels serve the packed 16-bit buckets of the 16-lane
// classes (the bulk of short-read work), split in two class ranges per mode
// so that the short classes run with more resident waves: part 0 holds
// classes 0..kPersistSmallMax, part 1 the classes up to kPersistMaxClass.
// The other buckets run as plain per-bucket launches after them.
#ifndef MICA_PERSIST_MAX_CLASS
#define MICA_PERSIST_MAX_CLASS 15
#endif
constexpr int kPersistSmallMax = 9;
constexpr int kPersistMaxClass = MICA_PERSIST_MAX_CLASS;
__host__ __device__ constexpr bool persistent_bucket(int b) {
  return bucket_kind(b) == kK16 && class_lanes(bucket_class(b)) == 16 && bucket_class(b) <= kPersistMaxClass;
}
__host__ __device__ constexpr int persist_part(int cls) { return cls <= kPersistSmallMax ? 0 : 1; }
// queue part of a persistent (mode, part): the long-read part of a mode
// first (its items cost most), then the short-read part
__host__ __device__ constexpr int persist_queue_part(int mode, int part) { return mode * 2 + (part ? 0 : 1); }
constexpr int kPersistParts = 2 * kNumModes;
constexpr int kQueueParts = kPersistParts + 1;  // the persistent parts, then everything else
// the ordering key of buckets in the work queue
__host__ __device__ constexpr int queue_part(int b) {
  return persistent_bucket(b) ? persist_queue_part(bucket_mode(b), persist_part(bucket_class(b))) : kPersistParts;
}

constexpr uint32_t kSkip = 0xFFFFFFFFu;

// counters[] slots
// (queue heads of the persistent kernels: kCtrQueueHead + queue part)
// (queue heads of the persistent side-list kernels: kCtrSideHead + queue part)
enum : int {
  kCtrQueueHead = 0,
  kCtrRerun = kPersistParts,
  kCtrItems,
  kCtrRerunHead,
  kCtrSideHead,
  kNumCounters = kCtrSideHead + kPersistParts
};

// per-pair status bits (same values as the public header)
constexpr uint32_t kStSaturated = 1u << 0;
constexpr uint32_t kStCigarTrunc = 1u << 1;
constexpr uint32_t kStLenLimit = 1u << 2;
constexpr uint32_t kStWinOob = 1u << 3;
constexpr uint32_t kStReadOob = 1u << 4;
constexpr uint32_t kStInternal = 1u << 5;

constexpr uint32_t kOutStart = 1u << 0;
constexpr uint32_t kOutCigar = 1u << 1;
constexpr uint32_t kForceInt32 = 1u << 8;

// LDS per wave (32-bit words): during the fill, a window-selector ring of 256
// columns for each of up to 4 lane groups; after it, the banded traceback's
// read and window codes in the same space.  The per-pair results (shifted score, i*, j*) and the
// extension's end-to-end candidates sit at the top.
constexpr int kRing = 256;
constexpr int kRingWords = 4 * kRing;
constexpr int kLdsWaveWords = 2048;
constexpr int kRedOff = kLdsWaveWords - 64;  // 8 pairs x 4 words
constexpr int kGslOff = kLdsWaveWords - 32;  // 8 pairs x 2 words
constexpr int kBandWords = kRedOff;          // band codes: [0, kRedOff)
static_assert(kRingWords <= kRedOff, "fill areas below the results");
constexpr int kWavesPerBlock = 4;
// widest band of the banded traceback (diagonals); wider pairs are traced
// back from a full fill of direction bits instead.  Bands up to
// kBandInlineW diagonals are refilled by the fill kernel (right after the
// fill, or in the 16-lane classes an item's worth at a time from the wave's
// pending list); wider ones by a later launch whose work items hold only
// such pairs.
constexpr int kBandMaxW = 64;
constexpr int kBandInlineW = 16;
// words at the end of a traceback slot that hold a wave's pending pairs
// (pairs whose band refill waits for an item's worth of them)
constexpr int kPendWords = 16;

struct Params {
  // batch (device pointers owned by the caller)
  const uint32_t* ref2b;
  uint64_t ref_len;
  const uint64_t* win_off;
  const int32_t* win_len;
  const uint32_t* reads2b;
  uint64_t reads_len;
  const uint64_t* read_off;
  const int32_t* read_len;
  const uint8_t* mode;
  int32_t default_mode;
  int32_t max_m, max_n;
  int32_t min_m;  // pairs with fewer read bases are rejected (a launch-planning bound)
  int64_t n_pairs;
  int32_t* score;
  int32_t* read_end;
  int32_t* ref_end;
  int32_t* read_start;
  int32_t* ref_start;
  uint32_t* cigar;
  int32_t cigar_cap;
  int32_t* n_cigar;
  uint32_t* status;
  int32_t sa, sb, so, se;  // match, mismatch, gap open, gap extend
  const int32_t* ext_h0;   // extension start score per pair (NULL: ext_default_h0)
  int32_t ext_default_h0;
  int32_t max_h0;          // largest extension start score accepted
  int32_t ext_clip;        // extension clipping penalty
  int32_t mode_mask;       // modes the batch may hold (bit per mode)
  uint32_t flags;
  // workspace (device memory of the context)
  uint32_t* bucket_of;         // [n_pairs] bucket * kSubBins + sub-bin, or kSkip
  uint32_t* sorted;            // [n_pairs] pair ids grouped by bucket, then sub-bin
  uint32_t* rerun;             // [n_pairs] pair ids to recompute with 32-bit scores
  uint32_t* bcount;            // [kNumBuckets]
  uint32_t* bstart;            // [kNumBuckets]
  uint32_t* scount;            // [kNumSubBuckets] pairs per (bucket, sub-bin)
  uint32_t* sfill;             // [kNumSubBuckets] next free position of each (bucket, sub-bin)
  uint32_t* qstart;            // [kNumBuckets + 1] first item of each queue position
  const uint32_t* qorder;      // [kNumBuckets] bucket served at each queue position
  const uint8_t* class_of_m;   // [kMaxM + 1]
  uint32_t* counters;          // [kNumCounters]
  uint32_t* bhead;             // [kNumBuckets] next work item of each plain bucket launch
  // The side lists of the banded fills: fb, pairs whose band was too wide
  // (full traceback); db, pairs with bands of 17-64 diagonals (refilled later)
  uint32_t* fbcount;           // [kNumBuckets] fb pairs per bucket
  uint32_t* fbsorted;          // [n_pairs] fb pairs, in their bucket's range of `sorted`
  uint32_t* fbqstart;          // [kNumBuckets + 1] first fb item of each queue position
  uint32_t* dbcount;           // [kNumBuckets] db pairs of 17-32 diagonals per bucket
  uint32_t* dbwide;            // [kNumBuckets] db pairs of 33-64 diagonals per bucket
  uint32_t* dbsorted;          // [n_pairs] db pairs in their bucket's range of `sorted`: 17-32
                               // diagonals from its start up, 33-64 from its end down
  uint32_t* dbqstart;          // [kNumBuckets + 1] first db item of each queue position
  uint32_t* sidehead;          // [kNumBuckets] next side-list item of each per-bucket side launch
  uint8_t* scratch;            // n_slots * slot_bytes
  uint64_t slot_bytes;         // per resident wave: direction bits + CIGAR staging
  uint64_t dir_bytes;          // direction-bit part of a slot
  int32_t stage_stride;        // CIGAR staging words per pair
  int32_t n_slots;             // resident waves the scratch is sized for
  uint32_t persist_q[kQueueParts];  // queue positions [persist_q[q], persist_q[q+1]) of queue part q
};

}  // namespace mica

namespace mica {
typedef void (*KernelFn)(const Params*);
// Kernel entry points of the library, indexed for the host runtime.
struct KernelTable {
  KernelFn bucket[2][kNumBuckets];  // [with traceback][bucket]
  KernelFn persistent[2][kNumModes][2];  // [with traceback][mode][class part]
  // the side lists after the banded fills: per bucket, and persistent over
  // the persistent buckets ([mode][class part]), after their item scan
  KernelFn side[kNumBuckets];
  KernelFn side_persistent[kNumModes][2];
  KernelFn sidescan;
  KernelFn rerun[2];
  KernelFn zero, plan, scan, scatter;
  KernelTable();
};
const KernelTable& kernels();
hipError_t launch_pack2bit(const uint8_t* codes, int64_t n, uint32_t* words, hipStream_t s);
}  // namespace mica
