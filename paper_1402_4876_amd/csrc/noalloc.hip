// Allocation-free entry point of the batch alignment
// (mica_dp_align_batch_noalloc): the same planning and fill kernels as
// mica_dp_align_batch, with every piece of device workspace a batch needs
// (parameter block, bucket tables and counters, plan table, per-pair work
// lists, traceback slots) carved out of one file-scope device array instead
// of context memory.  No call allocates or frees device memory and no HIP
// graph is built; the kernels are launched one by one on the caller's
// stream.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <mutex>

#include "ctx.h"
#include "dp_common.h"
#include "mica_dp.h"
#include "plan.h"

using namespace mica;

namespace {

constexpr size_t kScratchBytes = MICA_NOALLOC_SCRATCH_BYTES;
constexpr int64_t kMaxPairs = MICA_NOALLOC_MAX_PAIRS;

constexpr size_t al256(size_t x) { return (x + 255) / 256 * 256; }
// layout of the array
constexpr size_t kOffParams = 0;
constexpr size_t kOffSmall = kOffParams + al256(sizeof(Params));
constexpr size_t kOffClass = kOffSmall + al256(small::kWords * 4);
constexpr size_t kOffPairs = kOffClass + al256(kMaxM + 1);  // bucket_of | sorted | rerun | fbsorted | dbsorted
constexpr size_t kOffSlots = kOffPairs + al256((size_t)kPairLists * kMaxPairs * 4);  // traceback slots
static_assert(kOffSlots + (size_t(64) << 20) <= kScratchBytes, "room for the traceback slots");
static_assert(sizeof(Params) % 4 == 0, "parameter block copied as words");

// Each GPU the library runs on holds its own copy of this array until the
// process ends.  Host code never uses the name itself as an address: the
// device address comes from hipGetSymbolAddress (kept per device below).
static __device__ __align__(256) uint8_t scratch[kScratchBytes];

// The parameter block and queue order travel as a kernel argument, so the
// host needs no staging memory for them.
struct SetupArgs {
  Params prm;
  uint32_t qorder[kNumBuckets];
};

__global__ __launch_bounds__(256) void k_noalloc_setup(const SetupArgs a, uint8_t* __restrict__ base) {
  const uint32_t* src = (const uint32_t*)&a.prm;
  uint32_t* prm = (uint32_t*)(base + kOffParams);
  for (int i = threadIdx.x; i < (int)(sizeof(Params) / 4); i += blockDim.x) prm[i] = src[i];
  uint32_t* qo = (uint32_t*)(base + kOffSmall) + small::kQorder;
  for (int i = threadIdx.x; i < kNumBuckets; i += blockDim.x) qo[i] = a.qorder[i];
  uint8_t* cls = base + kOffClass;
  for (int m = threadIdx.x; m <= kMaxM; m += blockDim.x) cls[m] = (uint8_t)default_class_of(m);
}

struct DeviceState {
  bool ready = false;
  uint8_t* base = nullptr;  // device address of `scratch` on this GPU
  int n_cu = 0;
};
constexpr int kMaxDevices = 64;
DeviceState g_dev[kMaxDevices];
std::mutex g_mu;

// Set-up, once per device, with that device current: the device address of
// the array and the compute-unit count.
mica_status_t device_state(int dev, DeviceState* out) {
  std::lock_guard<std::mutex> g(g_mu);
  DeviceState& d = g_dev[dev];
  if (!d.ready) {
    void* p = nullptr;
    HIP_TRY(hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)));
    if (!p) return fail(MICA_ERR_HIP, "hipGetSymbolAddress gave no address for the fixed scratch");
    int ncu = 0;
    HIP_TRY(hipDeviceGetAttribute(&ncu, hipDeviceAttributeMultiprocessorCount, dev));
    d.base = (uint8_t*)p;
    d.n_cu = std::max(ncu, 1);
    d.ready = true;
  }
  *out = d;
  return MICA_OK;
}

hipError_t launch(KernelFn fn, unsigned blocks, unsigned threads, size_t shmem, hipStream_t s, const Params* dp) {
  void* args[] = {(void*)&dp};
  return hipLaunchKernel((const void*)fn, dim3(blocks), dim3(threads), args, shmem, s);
}

}  // namespace

extern "C" {

mica_status_t mica_dp_align_batch_noalloc(const mica_batch_t* b, const mica_scoring_t* s, uint32_t flags,
                                          void* stream_) {
  const uint32_t known = MICA_OUT_START | MICA_OUT_CIGAR | MICA_FORCE_INT32 | MICA_PLAIN_LAUNCH | MICA_NO_GRAPH;
  mica_status_t st = check_batch(b, s, flags, known);
  if (st != MICA_OK) return st;
  if (b->n_pairs > kMaxPairs)
    return fail(MICA_ERR_LIMIT, "more pairs than the allocation-free call takes (4,194,304)");
  if (b->n_pairs == 0) return MICA_OK;
  hipStream_t stream = (hipStream_t)stream_;
  int dev = 0;
  HIP_TRY(hipGetDevice(&dev));
  if (dev < 0 || dev >= kMaxDevices) return fail(MICA_ERR_INVALID_ARG, "device index beyond 63");
  DeviceState ds;
  st = device_state(dev, &ds);
  if (st != MICA_OK) return st;

  // the default plan (the same table the setup kernel writes to the device)
  uint8_t class_of_m[kMaxM + 1];
  for (int m = 0; m <= kMaxM; ++m) class_of_m[m] = (uint8_t)default_class_of(m);
  FillPlan fp;
  st = plan_fills(dev, class_of_m, b, s, flags, &fp);
  if (st != MICA_OK) return st;

  // resident waves: as many as the most occupant fill kernel keeps, as the
  // work needs, and as the slot area holds (whole blocks)
  const SlotShape sh = slot_shape(b, flags);
  const size_t area = kScratchBytes - kOffSlots;
  int64_t slots = (int64_t)fp.occ_max * ds.n_cu * kWavesPerBlock;
  const int64_t need = (b->n_pairs + 1) / 2 + 3;  // upper bound of work items
  slots = std::min<int64_t>(slots, (int64_t)align_up((size_t)need, kWavesPerBlock));
  slots = std::min<int64_t>(slots, (int64_t)(area / sh.slot_bytes) / kWavesPerBlock * kWavesPerBlock);
  if (slots < kWavesPerBlock)
    return fail(MICA_ERR_LIMIT, "windows too long for the allocation-free call's traceback slots");

  SetupArgs a;
  batch_params(&a.prm, b, s, flags, fp.mode_mask);
  Params& P = a.prm;
  uint32_t* sm = (uint32_t*)(ds.base + kOffSmall);
  uint32_t* pairs = (uint32_t*)(ds.base + kOffPairs);
  P.bucket_of = pairs;
  P.sorted = pairs + kMaxPairs;
  P.rerun = pairs + 2 * kMaxPairs;
  P.fbsorted = pairs + 3 * kMaxPairs;
  P.fbcount = sm + small::kFbcount;
  P.sidehead = sm + small::kSidehead;
  P.fbqstart = sm + small::kFbqstart;
  P.dbsorted = pairs + 4 * kMaxPairs;
  P.dbcount = sm + small::kDbcount;
  P.dbwide = sm + small::kDbwide;
  P.dbqstart = sm + small::kDbqstart;
  P.bcount = sm + small::kBcount;
  P.bstart = sm + small::kBstart;
  P.scount = sm + small::kScount;
  P.sfill = sm + small::kSfill;
  P.qstart = sm + small::kQstart;
  P.qorder = sm + small::kQorder;
  P.class_of_m = ds.base + kOffClass;
  P.counters = sm + small::kCounters;
  P.bhead = sm + small::kBhead;
  P.scratch = ds.base + kOffSlots;
  P.slot_bytes = sh.slot_bytes;
  P.dir_bytes = sh.dir_bytes;
  P.stage_stride = sh.stage_stride;
  P.n_slots = (int32_t)slots;
  queue_order(a.qorder, P.persist_q);
  const Params* dp = (const Params*)(ds.base + kOffParams);

  hipLaunchKernelGGL(k_noalloc_setup, dim3(1), dim3(256), 0, stream, a, ds.base);
  HIP_TRY(hipGetLastError());
  const KernelTable& K = kernels();
  const unsigned pblocks = (unsigned)((b->n_pairs + kPlanPairsPerBlock - 1) / kPlanPairsPerBlock);
  HIP_TRY(launch(K.zero, 1, 256, 0, stream, dp));
  HIP_TRY(launch(K.plan, pblocks, kPlanThreads, 0, stream, dp));
  HIP_TRY(launch(K.scan, 1, 256, 0, stream, dp));
  HIP_TRY(launch(K.scatter, pblocks, kPlanThreads, 0, stream, dp));
  for (int i = 0; i < fp.n; ++i) {
    const int64_t blocks = std::min<int64_t>((int64_t)fp.occ[i] * ds.n_cu, slots / kWavesPerBlock);
    if (fp.single[i]) HIP_TRY(launch(fp.fn[i], 1, 256, 0, stream, dp));
    else HIP_TRY(launch(fp.fn[i], (unsigned)std::max<int64_t>(blocks, 1), 256, kFillShmem, stream, dp));
  }
  return MICA_OK;
}

}  // extern "C"
