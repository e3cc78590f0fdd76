// Measured integer VALU throughput of the device: the roof the DP fill
// kernels are bound by.  Every lane of many resident waves runs eight
// independent chains of add and max instructions (the operations of the
// DP recurrence) on packed 16-bit pairs, or on 32-bit values; the rate is
// lane operations per second, a packed instruction counting two.
#include <hip/hip_runtime.h>

#include <string>

#include "ctx.h"
#include "mica_dp.h"

using namespace mica;

namespace {

constexpr int kChains = 8;
constexpr int kUnroll = 8;  // instructions per chain per loop iteration

template <bool PK>
__global__ __launch_bounds__(256) void k_valu_peak(uint32_t* __restrict__ out, int iters, uint32_t k) {
  uint32_t a[kChains];
#pragma unroll
  for (int i = 0; i < kChains; ++i) a[i] = threadIdx.x * 0x9E3779B9u + (uint32_t)i * 0x01000193u + blockIdx.x;
  for (int it = 0; it < iters; ++it) {
#pragma unroll
    for (int u = 0; u < kUnroll; ++u) {
#pragma unroll
      for (int i = 0; i < kChains; ++i) {
        if constexpr (PK) {
          if (u & 1) asm volatile("v_pk_max_i16 %0, %0, %1" : "+v"(a[i]) : "v"(k));
          else asm volatile("v_pk_add_u16 %0, %0, %1" : "+v"(a[i]) : "v"(k));
        } else {
          if (u & 1) asm volatile("v_max_i32 %0, %0, %1" : "+v"(a[i]) : "v"(k));
          else asm volatile("v_add_u32 %0, %0, %1" : "+v"(a[i]) : "v"(k));
        }
      }
    }
  }
  uint32_t x = 0;
#pragma unroll
  for (int i = 0; i < kChains; ++i) x ^= a[i];
  out[(size_t)blockIdx.x * blockDim.x + threadIdx.x] = x;
}

template <bool PK>
mica_status_t time_peak(int n_cu, uint32_t* d_out, hipEvent_t e0, hipEvent_t e1, double* tops) {
  const int blocks = n_cu * 8;  // 32 waves per CU, 8 per SIMD
  const int iters = 4096;
  hipLaunchKernelGGL(k_valu_peak<PK>, dim3(blocks), dim3(256), 0, nullptr, d_out, 64, 3u);
  HIP_TRY(hipGetLastError());
  HIP_TRY(hipEventRecord(e0, nullptr));
  hipLaunchKernelGGL(k_valu_peak<PK>, dim3(blocks), dim3(256), 0, nullptr, d_out, iters, 3u);
  HIP_TRY(hipGetLastError());
  HIP_TRY(hipEventRecord(e1, nullptr));
  HIP_TRY(hipEventSynchronize(e1));
  float ms = 0;
  HIP_TRY(hipEventElapsedTime(&ms, e0, e1));
  const double ops = (double)blocks * 256.0 * iters * kUnroll * kChains * (PK ? 2.0 : 1.0);
  *tops = ms > 0 ? ops / (ms * 1e-3) / 1e12 : 0.0;
  return MICA_OK;
}

}  // namespace

extern "C" {

mica_status_t mica_measure_valu_peak(int hip_device, double* tops_i16x2, double* tops_i32) {
  if (!tops_i16x2 || !tops_i32) return fail(MICA_ERR_INVALID_ARG, "NULL output");
  int ndev = 0;
  HIP_TRY(hipGetDeviceCount(&ndev));
  if (hip_device < 0 || hip_device >= ndev) return fail(MICA_ERR_INVALID_ARG, "no such HIP device");
  HIP_TRY(hipSetDevice(hip_device));
  int n_cu = 0;
  HIP_TRY(hipDeviceGetAttribute(&n_cu, hipDeviceAttributeMultiprocessorCount, hip_device));
  uint32_t* d_out = nullptr;
  HIP_TRY(hipMalloc(&d_out, (size_t)n_cu * 8 * 256 * sizeof(uint32_t)));
  hipEvent_t e0 = nullptr, e1 = nullptr;
  mica_status_t st = MICA_OK;
  if (hipEventCreate(&e0) != hipSuccess || hipEventCreate(&e1) != hipSuccess)
    st = fail(MICA_ERR_HIP, "hipEventCreate failed");
  if (st == MICA_OK) st = time_peak<true>(n_cu, d_out, e0, e1, tops_i16x2);
  if (st == MICA_OK) st = time_peak<false>(n_cu, d_out, e0, e1, tops_i32);
  if (e0) (void)hipEventDestroy(e0);
  if (e1) (void)hipEventDestroy(e1);
  (void)hipFree(d_out);
  return st;
}

}  // extern "C"
