// Host-side state of a library context, shared by the runtime's translation
// units (launch path, autotuner).  Not part of the public C ABI.
#pragma once
#include <hip/hip_runtime.h>

#include <map>
#include <string>
#include <utility>
#include <vector>

#include "dp_common.h"
#include "mica_dp.h"

namespace mica {

// record `msg` as this thread's last error text and return `st`
mica_status_t fail(mica_status_t st, const std::string& msg);

#define HIP_TRY(expr)                                                                       \
  do {                                                                                      \
    hipError_t e_ = (expr);                                                                 \
    if (e_ != hipSuccess)                                                                   \
      return ::mica::fail(MICA_ERR_HIP, std::string(#expr) + ": " + hipGetErrorString(e_)); \
  } while (0)

constexpr int kParamRing = 32;
constexpr size_t kDefaultWorkspace = size_t(8) << 30;

inline size_t align_up(size_t x, size_t a) { return (x + a - 1) / a * a; }

// Layout of the small device table area of a batch (bucket tables, queue
// order and counters), in 32-bit words.
namespace small {
constexpr size_t kBcount = 0;
constexpr size_t kBstart = kNumBuckets;
constexpr size_t kQstart = 2 * kNumBuckets;  // kNumBuckets + 1 entries
constexpr size_t kQorder = 3 * kNumBuckets + 8;
constexpr size_t kCounters = 4 * kNumBuckets + 8;
constexpr size_t kBhead = 4 * kNumBuckets + 8 + kNumCounters;
constexpr size_t kScount = 5 * kNumBuckets + 8 + kNumCounters;
constexpr size_t kSfill = kScount + kNumSubBuckets;
constexpr size_t kFbcount = kSfill + kNumSubBuckets;
constexpr size_t kSidehead = kFbcount + kNumBuckets;
constexpr size_t kFbqstart = kSidehead + kNumBuckets;  // kNumBuckets + 1 entries
constexpr size_t kDbcount = kFbqstart + kNumBuckets + 8;
constexpr size_t kDbwide = kDbcount + kNumBuckets;
constexpr size_t kDbqstart = kDbwide + kNumBuckets;  // kNumBuckets + 1 entries
constexpr size_t kWords = kDbqstart + kNumBuckets + 8;
}  // namespace small

// Work-queue order of the buckets (persistent parts first, each by
// descending item cost) and the queue positions where each persistent part
// starts (persist_q[q] .. persist_q[q + 1]).
void queue_order(uint32_t qorder[kNumBuckets], uint32_t persist_q[kQueueParts]);

// Validation of a batch and its flags shared by the batch entry points:
// MICA_OK or the batch-level error (with its text recorded).
mica_status_t check_batch(const mica_batch_t* b, const mica_scoring_t* s, uint32_t flags, uint32_t known_flags);

// The fill launches of a batch, in launch order, and the resident blocks per
// CU of each (its occupancy at the library's block shape).
constexpr int kMaxFills = 4 * kNumModes + 2 * kNumBuckets + 2;
// per-pair work lists of a batch: bucket_of | sorted | rerun | fbsorted | dbsorted
constexpr int kPairLists = 5;
struct FillPlan {
  KernelFn fn[kMaxFills];
  int occ[kMaxFills];
  bool single[kMaxFills];  // one block of 256 threads without dynamic LDS (a scan between fills)
  int n = 0;
  int occ_max = 1;
  int mode_mask = 0;  // modes the batch holds
};
mica_status_t plan_fills(int device, const uint8_t* class_of_m, const mica_batch_t* b, const mica_scoring_t* s,
                         uint32_t flags, FillPlan* out);

// Resident blocks per CU of a fill kernel (cached per device and kernel; no
// device memory is allocated).
mica_status_t kernel_occupancy(int device, KernelFn fn, int* blocks);

// Bytes of one resident wave's scratch slot (direction words + CIGAR
// staging) and its direction-word part; CIGAR staging words per pair.
struct SlotShape {
  size_t slot_bytes = 256, dir_bytes = 0;
  int stage_stride = 0;
};
SlotShape slot_shape(const mica_batch_t* b, uint32_t flags);

// LDS bytes of a fill block
constexpr size_t kFillShmem = (size_t)kWavesPerBlock * kLdsWaveWords * 4;

// The parameter block of a batch, without its workspace pointers.
void batch_params(Params* P, const mica_batch_t* b, const mica_scoring_t* s, uint32_t flags, int mode_mask);

// default plan: 16 lanes with the fewest rows that cover m, 64 x 16 above 256
__host__ __device__ constexpr int default_class_of(int m) {
  return m <= 256 ? (m == 0 ? 0 : (m + 15) / 16 - 1) : 16;
}

}  // namespace mica

struct mica_ctx {
  int device = 0;
  std::string arch;  // gcnArchName of the device
  size_t ws_cap = mica::kDefaultWorkspace;
  int n_cu = 256;
  // device memory
  mica::Params* d_params = nullptr;     // ring of kParamRing parameter blocks
  uint32_t* d_small = nullptr;    // bucket tables and counters
  uint8_t* d_class = nullptr;     // class_of_m
  uint32_t* d_pairs = nullptr;    // bucket_of | sorted | rerun
  int64_t pair_cap = 0;
  uint8_t* d_scratch = nullptr;
  size_t scratch_cap = 0;
  // host state
  mica::Params* h_params = nullptr;     // pinned ring
  hipEvent_t ev[mica::kParamRing] = {};
  bool ev_used[mica::kParamRing] = {};
  int ring_pos = 0;
  uint8_t class_of_m[mica::kMaxM + 1];
  uint32_t qorder[mica::kNumBuckets];
  uint32_t persist_q[mica::kQueueParts] = {};
  bool class_dirty = true;
  // fill-kernel timing
  bool timing = false;
  std::vector<hipEvent_t> ev_pool;
  std::vector<std::pair<hipEvent_t, hipEvent_t>> ev_pending;
  // launch graphs, one per launch sequence (kernel, block size and LDS of
  // every launch, and whether timing events are recorded); grid sizes and the
  // parameter block are set on the instantiated graph before each launch
  struct Graph {
    hipGraph_t graph = nullptr;
    hipGraphExec_t exec = nullptr;
    std::vector<hipGraphNode_t> kernel_nodes;
    hipGraphNode_t ev_begin = nullptr, ev_end = nullptr;
  };
  std::map<std::vector<uint64_t>, Graph> graphs;
  int64_t graph_launches = 0, graph_builds = 0;
  // last batch
  int64_t last_pairs = 0;
  int last_slots = 0;
  size_t last_scratch = 0;
};

