// Per-bucket fill kernels: 32-bit scores, semi-global, score and end cell only.
#include "dp_fill.h"

namespace mica {
void reg_fill_k32_0_0(KernelTable& t) {
  fill_bucket_table<kTbNone, kK32, 0>(t.bucket[0], ClassSeq{});
}
}  // namespace mica
