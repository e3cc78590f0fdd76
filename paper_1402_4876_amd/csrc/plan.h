// Launch shape of the planning kernels (k_plan, k_scatter), shared by the
// kernels and the host runtime that launches them.
#pragma once

namespace mica {
// threads per block, and pairs per thread: the per-block LDS histograms
// (every bucket and length bin) are cleared and flushed once per
// kPlanThreads * kPlanPairsPerThread pairs
constexpr int kPlanThreads = 256;
constexpr int kPlanPairsPerThread = 4;
constexpr int kPlanPairsPerBlock = kPlanThreads * kPlanPairsPerThread;
}  // namespace mica
