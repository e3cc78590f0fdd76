// Host runtime of the DP-phase library: context, argument validation, device
// workspace, kernel plan table and the launch sequence behind the C ABI.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstdio>
#include <cstring>
#include <map>
#include <mutex>
#include <string>
#include <utility>
#include <vector>

#include "ctx.h"
#include "dp_common.h"
#include "mica_dp.h"
#include "plan.h"

using namespace mica;

namespace mica {
thread_local std::string g_last_error;
mica_status_t fail(mica_status_t st, const std::string& msg) {
  g_last_error = msg;
  return st;
}
}  // namespace mica

namespace {
double bucket_cost(int b);
}

namespace mica {

void queue_order(uint32_t qorder[kNumBuckets], uint32_t persist_q[kQueueParts]) {
  int order[kNumBuckets];
  for (int b = 0; b < kNumBuckets; ++b) order[b] = b;
  // buckets of the persistent kernels first (per mode, long-read part
  // first), each part by descending item cost, then the plain buckets
  std::stable_sort(order, order + kNumBuckets, [](int x, int y) {
    if (queue_part(x) != queue_part(y)) return queue_part(x) < queue_part(y);
    return bucket_cost(x) > bucket_cost(y);
  });
  for (int q = 0; q < kQueueParts; ++q) persist_q[q] = 0;
  for (int b = 0; b < kNumBuckets; ++b)
    for (int q = queue_part(b); q + 1 < kQueueParts; ++q) persist_q[q + 1]++;
  for (int q = 0; q < kNumBuckets; ++q) qorder[q] = (uint32_t)order[q];
}

}  // namespace mica

namespace {

uint32_t* small_bcount(mica_ctx* c) { return c->d_small + small::kBcount; }
uint32_t* small_bstart(mica_ctx* c) { return c->d_small + small::kBstart; }
uint32_t* small_qstart(mica_ctx* c) { return c->d_small + small::kQstart; }
uint32_t* small_qorder(mica_ctx* c) { return c->d_small + small::kQorder; }
uint32_t* small_counters(mica_ctx* c) { return c->d_small + small::kCounters; }
uint32_t* small_bhead(mica_ctx* c) { return c->d_small + small::kBhead; }
uint32_t* small_scount(mica_ctx* c) { return c->d_small + small::kScount; }
uint32_t* small_sfill(mica_ctx* c) { return c->d_small + small::kSfill; }
uint32_t* small_fbcount(mica_ctx* c) { return c->d_small + small::kFbcount; }
uint32_t* small_sidehead(mica_ctx* c) { return c->d_small + small::kSidehead; }
constexpr size_t kSmallWords = small::kWords;

// cost of one work item of a bucket, for the descending work-queue order
double bucket_cost(int b) {
  const int kind = bucket_kind(b), cls = bucket_class(b), mode = bucket_mode(b);
  double c = class_rows(cls) * (class_lanes(cls) == 64 ? 1.5 : 1.0);
  if (mode == 1) c *= 1.25;
  if (kind == kK16Sat) c *= 1.1;
  if (kind == kK32) c *= 1.05;
  return c;
}

void default_plan(mica_ctx* c) {
  for (int m = 0; m <= kMaxM; ++m) c->class_of_m[m] = (uint8_t)default_class_of(m);
  c->class_dirty = true;
}

// same bounds as the device planner: can every cell stay inside int16?
// (extensions: start scores up to max_h0)
bool int16_always_safe(int max_m, int max_n, const mica_scoring_t& s, bool any_local, bool any_sg, bool any_ext,
                       int max_h0) {
  long hi = (long)s.match * (long)std::min(max_m, max_n);
  long lo = 0;
  if (any_sg) lo = std::min(lo, -(long)(2 * s.gap_open + (long)(max_m + 1) * s.gap_extend) - (kMaxM - 1));
  if (any_local) lo = std::min(lo, -(long)(s.gap_open + s.gap_extend) - (kMaxM - 1));
  if (any_ext) {
    hi = std::max(hi, (long)max_h0 + (long)s.match * (long)std::min(max_m, max_n));
    lo = std::min(lo, -3L * s.gap_open - (long)(max_m + max_n + 1) * s.gap_extend);
  }
  return hi <= 32767 - 8 && lo >= -32767 + 8;
}

mica_status_t ensure_pairs(mica_ctx* c, int64_t n) {
  if (n <= c->pair_cap) return MICA_OK;
  if (c->d_pairs) HIP_TRY(hipFree(c->d_pairs));
  c->d_pairs = nullptr;
  const int64_t cap = std::max<int64_t>(n, 1024);
  if (hipMalloc(&c->d_pairs, (size_t)cap * kPairLists * sizeof(uint32_t)) != hipSuccess) {
    c->pair_cap = 0;
    return fail(MICA_ERR_OUT_OF_MEMORY, "cannot allocate per-pair workspace");
  }
  c->pair_cap = cap;
  return MICA_OK;
}

mica_status_t ensure_scratch(mica_ctx* c, size_t bytes) {
  if (bytes <= c->scratch_cap) return MICA_OK;
  if (c->d_scratch) HIP_TRY(hipFree(c->d_scratch));
  c->d_scratch = nullptr;
  if (hipMalloc(&c->d_scratch, bytes) != hipSuccess) {
    c->scratch_cap = 0;
    return fail(MICA_ERR_OUT_OF_MEMORY, "cannot allocate traceback scratch");
  }
  c->scratch_cap = bytes;
  return MICA_OK;
}

hipError_t take_event(mica_ctx* c, hipEvent_t* e) {
  if (!c->ev_pool.empty()) {
    *e = c->ev_pool.back();
    c->ev_pool.pop_back();
    return hipSuccess;
  }
  return hipEventCreate(e);
}

hipError_t launch(KernelFn fn, unsigned blocks, unsigned threads, size_t shmem, hipStream_t s,
                  const Params* dp) {
  void* args[] = {(void*)&dp};
  return hipLaunchKernel((const void*)fn, dim3(blocks), dim3(threads), args, shmem, s);
}

// One kernel launch of a batch; `fill` marks the launches the timing events
// bracket.
struct Launch {
  KernelFn fn;
  unsigned grid, block;
  size_t shmem;
  bool fill;
};

hipKernelNodeParams node_params(const Launch& l, void** args) {
  hipKernelNodeParams p;
  std::memset(&p, 0, sizeof(p));
  p.func = (void*)l.fn;
  p.gridDim = dim3(l.grid);
  p.blockDim = dim3(l.block);
  p.sharedMemBytes = (unsigned)l.shmem;
  p.kernelParams = args;
  p.extra = nullptr;
  return p;
}

// Build the graph of a launch sequence: a chain of kernel nodes, with event
// record nodes around the fill launches when timing is on.
mica_status_t build_graph(mica_ctx* c, const std::vector<Launch>& seq, bool timing, const Params* dp,
                          hipEvent_t t0, hipEvent_t t1, mica_ctx::Graph* out) {
  mica_ctx::Graph g;
  HIP_TRY(hipGraphCreate(&g.graph, 0));
  hipGraphNode_t prev = nullptr;
  auto add_event = [&](hipEvent_t e, hipGraphNode_t* node) -> hipError_t {
    hipError_t err = hipGraphAddEventRecordNode(node, g.graph, prev ? &prev : nullptr, prev ? 1 : 0, e);
    if (err == hipSuccess) prev = *node;
    return err;
  };
  bool began = false;
  for (size_t i = 0; i < seq.size(); ++i) {
    if (timing && seq[i].fill && !began) {
      HIP_TRY(add_event(t0, &g.ev_begin));
      began = true;
    }
    void* args[] = {(void*)&dp};
    hipKernelNodeParams p = node_params(seq[i], args);
    hipGraphNode_t node;
    HIP_TRY(hipGraphAddKernelNode(&node, g.graph, prev ? &prev : nullptr, prev ? 1 : 0, &p));
    g.kernel_nodes.push_back(node);
    prev = node;
    const bool last_fill = seq[i].fill && (i + 1 == seq.size() || !seq[i + 1].fill);
    if (timing && last_fill) HIP_TRY(add_event(t1, &g.ev_end));
  }
  if (timing && !began) {  // no fill launch: the two events are adjacent
    HIP_TRY(add_event(t0, &g.ev_begin));
    HIP_TRY(add_event(t1, &g.ev_end));
  }
  HIP_TRY(hipGraphInstantiate(&g.exec, g.graph, nullptr, nullptr, 0));
  c->graph_builds++;
  *out = g;
  return MICA_OK;
}

mica_status_t run_sequence(mica_ctx* c, const std::vector<Launch>& seq, const Params* dp, hipStream_t stream,
                           bool use_graph, hipEvent_t t0, hipEvent_t t1) {
  const bool timing = t0 != nullptr;
  if (!use_graph) {
    bool began = false;
    for (size_t i = 0; i < seq.size(); ++i) {
      if (timing && seq[i].fill && !began) {
        HIP_TRY(hipEventRecord(t0, stream));
        began = true;
      }
      HIP_TRY(launch(seq[i].fn, seq[i].grid, seq[i].block, seq[i].shmem, stream, dp));
      if (timing && seq[i].fill && (i + 1 == seq.size() || !seq[i + 1].fill)) HIP_TRY(hipEventRecord(t1, stream));
    }
    if (timing && !began) {
      HIP_TRY(hipEventRecord(t0, stream));
      HIP_TRY(hipEventRecord(t1, stream));
    }
    return MICA_OK;
  }
  std::vector<uint64_t> key;
  key.push_back(timing ? 1 : 0);
  for (const Launch& l : seq) {
    key.push_back((uint64_t)(uintptr_t)l.fn);
    key.push_back(((uint64_t)l.block << 32) | (uint64_t)l.shmem);
    key.push_back(l.fill ? 1 : 0);
  }
  auto it = c->graphs.find(key);
  if (it == c->graphs.end()) {
    mica_ctx::Graph g;
    mica_status_t st = build_graph(c, seq, timing, dp, t0, t1, &g);
    if (st != MICA_OK) return st;
    it = c->graphs.emplace(std::move(key), g).first;
  } else {
    mica_ctx::Graph& g = it->second;
    for (size_t i = 0; i < seq.size(); ++i) {
      void* args[] = {(void*)&dp};
      hipKernelNodeParams p = node_params(seq[i], args);
      HIP_TRY(hipGraphExecKernelNodeSetParams(g.exec, g.kernel_nodes[i], &p));
    }
    if (timing) {
      HIP_TRY(hipGraphExecEventRecordNodeSetEvent(g.exec, g.ev_begin, t0));
      HIP_TRY(hipGraphExecEventRecordNodeSetEvent(g.exec, g.ev_end, t1));
    }
  }
  HIP_TRY(hipGraphLaunch(it->second.exec, stream));
  c->graph_launches++;
  return MICA_OK;
}

}  // namespace

namespace mica {

mica_status_t check_batch(const mica_batch_t* b, const mica_scoring_t* s, uint32_t flags, uint32_t known) {
  if (!b || !s) return fail(MICA_ERR_INVALID_ARG, "NULL batch or scoring");
  if (flags & ~known) return fail(MICA_ERR_INVALID_ARG, "unknown flag bits");
  if (s->match < 1 || s->match > 4096 || s->mismatch > 0 || s->mismatch < -4096 || s->gap_open < 0 ||
      s->gap_open > 4096 || s->gap_extend < 1 || s->gap_extend > 4096)
    return fail(MICA_ERR_INVALID_ARG, "scoring outside its limits");
  if (b->n_pairs < 0) return fail(MICA_ERR_INVALID_ARG, "n_pairs < 0");
  if (b->n_pairs > 0xFFFFFFF0ll) return fail(MICA_ERR_LIMIT, "too many pairs in one batch");
  if (b->default_mode < 0 || b->default_mode > 2) return fail(MICA_ERR_INVALID_ARG, "bad default_mode");
  if (b->mode_mask < 0 || b->mode_mask > 7) return fail(MICA_ERR_INVALID_ARG, "bad mode_mask");
  if (b->ext_clip < 0 || b->ext_clip > kMaxH0 || b->ext_default_h0 < 0 || b->ext_default_h0 > kMaxH0)
    return fail(MICA_ERR_INVALID_ARG, "extension start score or clipping penalty outside 0..2^20");
  if (b->max_read_len < 0 || b->max_read_len > kMaxM || b->max_win_len < 0 || b->max_win_len > kMaxN)
    return fail(MICA_ERR_LIMIT, "max_read_len / max_win_len beyond the library limits");
  if (b->min_read_len < 0 || b->min_read_len > b->max_read_len)
    return fail(MICA_ERR_INVALID_ARG, "min_read_len outside [0, max_read_len]");
  if (b->max_ext_h0 < 0 || b->max_ext_h0 > kMaxH0)
    return fail(MICA_ERR_INVALID_ARG, "max_ext_h0 outside 0..2^20");
  const bool want_cigar = flags & MICA_OUT_CIGAR;
  const bool want_start = want_cigar || (flags & MICA_OUT_START);
  if (b->n_pairs == 0) return MICA_OK;
  if (!b->ref2b || !b->win_off || !b->win_len || !b->reads2b || !b->read_off || !b->read_len ||
      !b->score || !b->read_end || !b->ref_end || !b->status)
    return fail(MICA_ERR_INVALID_ARG, "NULL input or output pointer");
  if (want_start && (!b->read_start || !b->ref_start))
    return fail(MICA_ERR_INVALID_ARG, "read_start / ref_start required for start or CIGAR output");
  if (want_cigar && (!b->n_cigar || b->cigar_cap < 0 || (b->cigar_cap > 0 && !b->cigar)))
    return fail(MICA_ERR_INVALID_ARG, "cigar / n_cigar / cigar_cap invalid");
  return MICA_OK;
}

namespace {
struct OccEntry {
  int device;
  KernelFn fn;
  int blocks;
};
constexpr int kOccCache = 1024;
OccEntry g_occ[kOccCache];
int g_n_occ = 0;
std::mutex g_occ_mu;
}  // namespace

mica_status_t kernel_occupancy(int device, KernelFn fn, int* blocks) {
  std::lock_guard<std::mutex> g(g_occ_mu);
  for (int i = 0; i < g_n_occ; ++i)
    if (g_occ[i].device == device && g_occ[i].fn == fn) {
      *blocks = g_occ[i].blocks;
      return MICA_OK;
    }
  int nb = 0;
  HIP_TRY(hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, (const void*)fn, 256, kFillShmem));
  nb = std::max(nb, 1);
  if (g_n_occ < kOccCache) g_occ[g_n_occ++] = {device, fn, nb};
  *blocks = nb;
  return MICA_OK;
}

mica_status_t plan_fills(int device, const uint8_t* class_of_m, const mica_batch_t* b, const mica_scoring_t* s,
                         uint32_t flags, FillPlan* out) {
  const KernelTable& K = kernels();
  FillPlan& fp = *out;
  fp.n = 0;
  for (int i = 0; i < kMaxFills; ++i) fp.single[i] = false;
  fp.occ_max = 1;
  const int max_m = b->max_read_len, max_n = b->max_win_len;
  const int d = (flags & (MICA_OUT_CIGAR | MICA_OUT_START)) ? 1 : 0;
  const bool forced = flags & MICA_FORCE_INT32;
  const int mode_mask = b->mode ? (b->mode_mask ? b->mode_mask : 7) : 1 << b->default_mode;
  fp.mode_mask = mode_mask;
  const bool any_sg = mode_mask & 1, any_local = mode_mask & 2, any_ext = mode_mask & 4;
  const bool any_mode[3] = {any_sg, any_local, any_ext};
  // extensions start from per-pair scores the host does not read: without
  // a bound on them their saturating variants are always available
  const bool may_sat = !forced && ((any_ext && b->max_ext_h0 == 0) ||
                                   !int16_always_safe(max_m, max_n, *s, any_local, any_sg, any_ext, b->max_ext_h0));
  const bool plain = flags & MICA_PLAIN_LAUNCH;
  bool cls_used[kNumClasses] = {};
  for (int m = std::max(1, b->min_read_len); m <= max_m; ++m) cls_used[class_of_m[m]] = true;
  // a batch of one persistent class gains nothing from the persistent
  // kernels (they balance classes against each other) and its plain kernel
  // is compiled for that class alone
  int n_persist_cls = 0;
  for (int cls = 0; cls <= kPersistMaxClass; ++cls)
    if (cls_used[cls] && class_lanes(cls) == 16) ++n_persist_cls;
  const bool persist = !plain && !forced && n_persist_cls > 1;
  bool part_used[2] = {false, false};
  for (int cls = 0; cls <= kPersistMaxClass; ++cls)
    if (cls_used[cls] && class_lanes(cls) == 16) part_used[persist_part(cls)] = true;
  if (persist) {
    // persistent parts in queue order: per mode, long reads first
    for (int md = 0; md < kNumModes; ++md) {
      if (!any_mode[md]) continue;
      for (int part : {1, 0})
        if (part_used[part]) fp.fn[fp.n++] = K.persistent[d][md][part];
    }
  }
  // plain launches: every bucket in plain mode, else the buckets the
  // persistent kernels do not serve
  auto plain_buckets = [&](const KernelFn* table) {
    for (int kind = 0; kind < kNumKinds; ++kind) {
      if (forced != (kind == kK32)) continue;
      if (kind == kK16Sat && !may_sat) continue;
      for (int cls = 0; cls < kNumClasses; ++cls) {
        if (!cls_used[cls]) continue;
        for (int md = 0; md < kNumModes; ++md) {
          if (!any_mode[md]) continue;
          const int bk = bucket_id(kind, cls, md);
          if (persist && persistent_bucket(bk)) continue;
          fp.fn[fp.n++] = table[bk];
        }
      }
    }
  };
  plain_buckets(K.bucket[d]);
  // the side lists of the banded fills (pairs whose band was too wide: the
  // full traceback; bands of 17-64 diagonals: the band refill), after every
  // banded fill: persistent kernels over the persistent buckets (one queue
  // per mode and class part) and one launch per other bucket
  if (d) {
    if (persist) {
      fp.single[fp.n] = true;
      fp.fn[fp.n++] = K.sidescan;
      for (int md = 0; md < kNumModes; ++md) {
        if (!any_mode[md]) continue;
        for (int part : {1, 0})
          if (part_used[part]) fp.fn[fp.n++] = K.side_persistent[md][part];
      }
    }
    plain_buckets(K.side);
  }
  if (may_sat) fp.fn[fp.n++] = K.rerun[d];
  for (int i = 0; i < fp.n; ++i) {
    if (fp.single[i]) {
      fp.occ[i] = 1;
      continue;
    }
    mica_status_t st = kernel_occupancy(device, fp.fn[i], &fp.occ[i]);
    if (st != MICA_OK) return st;
    fp.occ_max = std::max(fp.occ_max, fp.occ[i]);
  }
  return MICA_OK;
}

SlotShape slot_shape(const mica_batch_t* b, uint32_t flags) {
  SlotShape sh;
  const int d = (flags & (MICA_OUT_CIGAR | MICA_OUT_START)) ? 1 : 0;
  // the full traceback's direction words (steps x 64 lanes x 16 B), or the
  // band records (two rows per word, 4 strips x 64 lanes), whichever is larger
  sh.dir_bytes = d ? std::max((size_t)(b->max_win_len + 64) * 64 * 16, (size_t)(b->max_read_len / 2 + 1) * 1024) : 0;
  sh.stage_stride = b->max_read_len + b->max_win_len + 2;
  // then a wave's pending pairs (kPendWords words)
  const size_t stage_bytes = d ? (size_t)8 * sh.stage_stride * 4 + kPendWords * 4 : 0;
  sh.slot_bytes = std::max<size_t>(align_up(sh.dir_bytes + stage_bytes, 256), 256);
  return sh;
}

void batch_params(Params* P_, const mica_batch_t* b, const mica_scoring_t* s, uint32_t flags, int mode_mask) {
  Params& P = *P_;
  const bool want_cigar = flags & MICA_OUT_CIGAR;
  const bool want_start = want_cigar || (flags & MICA_OUT_START);
  std::memset(&P, 0, sizeof(P));
  P.ref2b = b->ref2b;
  P.ref_len = b->ref_len;
  P.win_off = b->win_off;
  P.win_len = b->win_len;
  P.reads2b = b->reads2b;
  P.reads_len = b->reads_len;
  P.read_off = b->read_off;
  P.read_len = b->read_len;
  P.mode = b->mode;
  P.default_mode = b->default_mode;
  P.ext_h0 = b->ext_h0;
  P.ext_default_h0 = b->ext_default_h0;
  P.max_h0 = b->max_ext_h0 ? b->max_ext_h0 : kMaxH0;
  P.ext_clip = b->ext_clip;
  P.mode_mask = mode_mask;
  P.max_m = b->max_read_len;
  P.min_m = b->min_read_len;
  P.max_n = b->max_win_len;
  P.n_pairs = b->n_pairs;
  P.score = b->score;
  P.read_end = b->read_end;
  P.ref_end = b->ref_end;
  P.read_start = want_start ? b->read_start : nullptr;
  P.ref_start = want_start ? b->ref_start : nullptr;
  P.cigar = want_cigar ? b->cigar : nullptr;
  P.cigar_cap = want_cigar ? b->cigar_cap : 0;
  P.n_cigar = want_cigar ? b->n_cigar : nullptr;
  P.status = b->status;
  P.sa = s->match;
  P.sb = s->mismatch;
  P.so = s->gap_open;
  P.se = s->gap_extend;
  P.flags = (want_start ? kOutStart : 0u) | (want_cigar ? kOutCigar : 0u) |
            ((flags & MICA_FORCE_INT32) ? kForceInt32 : 0u);
}

}  // namespace mica

extern "C" {

const char* mica_last_error(void) { return g_last_error.c_str(); }

mica_status_t mica_ctx_create(int hip_device, size_t workspace_bytes, mica_ctx_t* out) {
  if (!out) return fail(MICA_ERR_INVALID_ARG, "out is NULL");
  *out = nullptr;
  int ndev = 0;
  HIP_TRY(hipGetDeviceCount(&ndev));
  if (hip_device < 0 || hip_device >= ndev) return fail(MICA_ERR_INVALID_ARG, "no such HIP device");
  HIP_TRY(hipSetDevice(hip_device));
  mica_ctx* c = new mica_ctx();
  c->device = hip_device;
  if (workspace_bytes) c->ws_cap = workspace_bytes;
  hipDeviceProp_t prop;
  HIP_TRY(hipGetDeviceProperties(&prop, hip_device));
  c->n_cu = prop.multiProcessorCount;
  c->arch = prop.gcnArchName;
  {
    const size_t colon = c->arch.find(':');
    if (colon != std::string::npos) c->arch.resize(colon);
  }
  HIP_TRY(hipMalloc(&c->d_params, sizeof(Params) * kParamRing));
  HIP_TRY(hipMalloc(&c->d_small, kSmallWords * sizeof(uint32_t)));
  HIP_TRY(hipMalloc(&c->d_class, kMaxM + 1));
  HIP_TRY(hipHostMalloc((void**)&c->h_params, sizeof(Params) * kParamRing, hipHostMallocDefault));
  for (int i = 0; i < kParamRing; ++i) HIP_TRY(hipEventCreateWithFlags(&c->ev[i], hipEventDisableTiming));
  default_plan(c);
  queue_order(c->qorder, c->persist_q);
  HIP_TRY(hipMemcpy(small_qorder(c), c->qorder, sizeof(c->qorder), hipMemcpyHostToDevice));
  HIP_TRY(hipMemcpy(c->d_class, c->class_of_m, kMaxM + 1, hipMemcpyHostToDevice));
  c->class_dirty = false;
  *out = c;
  return MICA_OK;
}

mica_status_t mica_ctx_destroy(mica_ctx_t c) {
  if (!c) return MICA_OK;
  (void)hipSetDevice(c->device);
  (void)hipDeviceSynchronize();
  for (int i = 0; i < kParamRing; ++i)
    if (c->ev[i]) (void)hipEventDestroy(c->ev[i]);
  if (c->h_params) (void)hipHostFree(c->h_params);
  if (c->d_params) (void)hipFree(c->d_params);
  if (c->d_small) (void)hipFree(c->d_small);
  if (c->d_class) (void)hipFree(c->d_class);
  if (c->d_pairs) (void)hipFree(c->d_pairs);
  if (c->d_scratch) (void)hipFree(c->d_scratch);
  for (auto& pr : c->ev_pending) {
    (void)hipEventDestroy(pr.first);
    (void)hipEventDestroy(pr.second);
  }
  for (auto e : c->ev_pool) (void)hipEventDestroy(e);
  for (auto& kv : c->graphs) {
    if (kv.second.exec) (void)hipGraphExecDestroy(kv.second.exec);
    if (kv.second.graph) (void)hipGraphDestroy(kv.second.graph);
  }
  delete c;
  return MICA_OK;
}

mica_status_t mica_ctx_set_plan(mica_ctx_t c, int32_t m_lo, int32_t m_hi, int32_t lanes, int32_t rows) {
  if (!c) return fail(MICA_ERR_INVALID_ARG, "ctx is NULL");
  if (m_lo < 1 || m_hi > kMaxM || m_lo > m_hi) return fail(MICA_ERR_INVALID_ARG, "bad read-length range");
  const int cls = class_of(lanes, rows);
  if (cls < 0) return fail(MICA_ERR_INVALID_ARG, "unsupported (lanes, rows)");
  if (lanes * rows < m_hi) return fail(MICA_ERR_INVALID_ARG, "lanes * rows must cover m_hi");
  HIP_TRY(hipSetDevice(c->device));
  // a batch still queued on any stream reads the device table when its
  // planning kernel runs, but its fill kernels were chosen from the host
  // table when it was enqueued: let every such batch finish first
  HIP_TRY(hipDeviceSynchronize());
  for (int m = m_lo; m <= m_hi; ++m) c->class_of_m[m] = (uint8_t)cls;
  HIP_TRY(hipMemcpy(c->d_class, c->class_of_m, kMaxM + 1, hipMemcpyHostToDevice));
  return MICA_OK;
}

mica_status_t mica_pack_2bit(const uint8_t* codes, int64_t n_bases, uint32_t* words, void* stream) {
  if (n_bases < 0) return fail(MICA_ERR_INVALID_ARG, "n_bases < 0");
  if (n_bases > 0 && (!codes || !words)) return fail(MICA_ERR_INVALID_ARG, "NULL pointer");
  HIP_TRY(launch_pack2bit(codes, n_bases, words, (hipStream_t)stream));
  return MICA_OK;
}

mica_status_t mica_dp_align_batch(mica_ctx_t c, const mica_batch_t* b, const mica_scoring_t* s,
                                  uint32_t flags, void* stream_) {
  if (!c) return fail(MICA_ERR_INVALID_ARG, "NULL ctx");
  const uint32_t known = MICA_OUT_START | MICA_OUT_CIGAR | MICA_FORCE_INT32 | MICA_PLAIN_LAUNCH | MICA_NO_GRAPH;
  mica_status_t st = check_batch(b, s, flags, known);
  if (st != MICA_OK) return st;
  if (b->n_pairs == 0) return MICA_OK;
  hipStream_t stream = (hipStream_t)stream_;
  HIP_TRY(hipSetDevice(c->device));

  st = ensure_pairs(c, b->n_pairs);
  if (st != MICA_OK) return st;

  // fill launches of this batch
  FillPlan fp;
  st = plan_fills(c->device, c->class_of_m, b, s, flags, &fp);
  if (st != MICA_OK) return st;

  // scratch: direction bits of a resident wave (steps x 64 lanes x 16 B) +
  // CIGAR staging, for as many waves as the most occupant fill kernel keeps
  // resident
  const SlotShape sh = slot_shape(b, flags);
  int64_t slots = (int64_t)fp.occ_max * c->n_cu * kWavesPerBlock;
  const int64_t by_ws = (int64_t)(c->ws_cap / sh.slot_bytes);
  slots = std::min(slots, by_ws);
  const int64_t need = (b->n_pairs + 1) / 2 + 3;  // upper bound of work items
  slots = std::min(slots, need);
  slots = std::max<int64_t>(align_up((size_t)std::max<int64_t>(slots, 1), kWavesPerBlock), kWavesPerBlock);
  if ((size_t)slots * sh.slot_bytes > c->ws_cap && slots > kWavesPerBlock)
    slots = (int64_t)(c->ws_cap / sh.slot_bytes) / kWavesPerBlock * kWavesPerBlock;
  if (slots < kWavesPerBlock) return fail(MICA_ERR_OUT_OF_MEMORY, "workspace too small for one block");
  st = ensure_scratch(c, (size_t)slots * sh.slot_bytes);
  if (st != MICA_OK) return st;

  // parameter block (pinned ring slot, copied on the stream)
  const int rp = c->ring_pos;
  c->ring_pos = (c->ring_pos + 1) % kParamRing;
  if (c->ev_used[rp]) HIP_TRY(hipEventSynchronize(c->ev[rp]));
  Params& P = c->h_params[rp];
  batch_params(&P, b, s, flags, fp.mode_mask);
  P.bucket_of = c->d_pairs;
  P.sorted = c->d_pairs + c->pair_cap;
  P.rerun = c->d_pairs + 2 * c->pair_cap;
  P.fbsorted = c->d_pairs + 3 * c->pair_cap;
  P.fbcount = small_fbcount(c);
  P.sidehead = small_sidehead(c);
  P.fbqstart = c->d_small + small::kFbqstart;
  P.dbsorted = c->d_pairs + 4 * c->pair_cap;
  P.dbcount = c->d_small + small::kDbcount;
  P.dbwide = c->d_small + small::kDbwide;
  P.dbqstart = c->d_small + small::kDbqstart;
  P.bcount = small_bcount(c);
  P.bstart = small_bstart(c);
  P.scount = small_scount(c);
  P.sfill = small_sfill(c);
  P.qstart = small_qstart(c);
  P.qorder = small_qorder(c);
  P.class_of_m = c->d_class;
  P.counters = small_counters(c);
  P.bhead = small_bhead(c);
  P.scratch = c->d_scratch;
  P.slot_bytes = sh.slot_bytes;
  P.dir_bytes = sh.dir_bytes;
  P.stage_stride = sh.stage_stride;
  P.n_slots = (int32_t)slots;
  for (int i = 0; i < kQueueParts; ++i) P.persist_q[i] = c->persist_q[i];
  Params* dp = c->d_params + rp;
  HIP_TRY(hipMemcpyAsync(dp, &P, sizeof(Params), hipMemcpyHostToDevice, stream));
  HIP_TRY(hipEventRecord(c->ev[rp], stream));
  c->ev_used[rp] = true;

  const KernelTable& K = kernels();
  const unsigned pblocks = (unsigned)((b->n_pairs + kPlanPairsPerBlock - 1) / kPlanPairsPerBlock);
  std::vector<Launch> seq;
  seq.push_back({K.zero, 1, 256, 0, false});
  seq.push_back({K.plan, pblocks, kPlanThreads, 0, false});
  seq.push_back({K.scan, 1, 256, 0, false});
  seq.push_back({K.scatter, pblocks, kPlanThreads, 0, false});
  for (int i = 0; i < fp.n; ++i) {
    // each fill kernel gets the blocks it keeps resident (its waves index
    // the first slots of the scratch)
    const int64_t blocks = std::min<int64_t>((int64_t)fp.occ[i] * c->n_cu, slots / kWavesPerBlock);
    if (fp.single[i]) seq.push_back({fp.fn[i], 1, 256, 0, true});
    else seq.push_back({fp.fn[i], (unsigned)std::max<int64_t>(blocks, 1), 256, kFillShmem, true});
  }
  hipEvent_t t0 = nullptr, t1 = nullptr;
  if (c->timing) {
    HIP_TRY(take_event(c, &t0));
    HIP_TRY(take_event(c, &t1));
  }
  st = run_sequence(c, seq, dp, stream, !(flags & MICA_NO_GRAPH), t0, t1);
  if (st != MICA_OK) return st;
  if (c->timing) c->ev_pending.emplace_back(t0, t1);
  c->last_pairs = b->n_pairs;
  c->last_slots = (int)slots;
  c->last_scratch = (size_t)slots * sh.slot_bytes;
  return MICA_OK;
}

mica_status_t mica_ctx_set_timing(mica_ctx_t c, int enable) {
  if (!c) return fail(MICA_ERR_INVALID_ARG, "ctx is NULL");
  c->timing = enable != 0;
  return MICA_OK;
}

mica_status_t mica_ctx_read_timing(mica_ctx_t c, double* fill_ms, int64_t* n_batches) {
  if (!c || !fill_ms || !n_batches) return fail(MICA_ERR_INVALID_ARG, "NULL argument");
  HIP_TRY(hipSetDevice(c->device));
  double total = 0;
  for (auto& pr : c->ev_pending) {
    HIP_TRY(hipEventSynchronize(pr.second));
    float ms = 0;
    HIP_TRY(hipEventElapsedTime(&ms, pr.first, pr.second));
    total += ms;
    c->ev_pool.push_back(pr.first);
    c->ev_pool.push_back(pr.second);
  }
  *fill_ms = total;
  *n_batches = (int64_t)c->ev_pending.size();
  c->ev_pending.clear();
  return MICA_OK;
}

mica_status_t mica_ctx_last_stats(mica_ctx_t c, void* stream, mica_batch_stats_t* out) {
  if (!c || !out) return fail(MICA_ERR_INVALID_ARG, "NULL argument");
  HIP_TRY(hipSetDevice(c->device));
  HIP_TRY(hipStreamSynchronize((hipStream_t)stream));
  uint32_t ctr[kNumCounters];
  HIP_TRY(hipMemcpy(ctr, small_counters(c), sizeof(ctr), hipMemcpyDeviceToHost));
  out->n_pairs = c->last_pairs;
  out->n_items = ctr[kCtrItems];
  out->n_saturated = ctr[kCtrRerun];
  out->n_waves = c->last_slots;
  out->scratch_bytes = (int64_t)c->last_scratch;
  uint32_t fbc[kNumBuckets];
  HIP_TRY(hipMemcpy(fbc, small_fbcount(c), sizeof(fbc), hipMemcpyDeviceToHost));
  out->n_fallback = 0;
  for (int b = 0; b < kNumBuckets; ++b) out->n_fallback += fbc[b];
  out->n_deferred = 0;
  for (size_t list : {small::kDbcount, small::kDbwide}) {
    HIP_TRY(hipMemcpy(fbc, c->d_small + list, sizeof(fbc), hipMemcpyDeviceToHost));
    for (int b = 0; b < kNumBuckets; ++b) out->n_deferred += fbc[b];
  }
  return MICA_OK;
}

}  // extern "C"
