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

// default plan: 16 lanes with the fewest rows that cover m, 64 x 16 above 256
inline int default_class_of(int m) { return m <= 256 ? (m == 0 ? 0 : (m + 15) / 16 - 1) : 16; }

}  // namespace mica

struct mica_ctx {
  int device = 0;
  std::string arch;  // gcnArchName of the device
  size_t ws_cap = mica::kDefaultWorkspace;
  int n_cu = 256;
  std::map<const void*, int> occ_cache;  // resident blocks per CU of each fill kernel
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

