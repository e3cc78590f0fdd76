// Per-bucket fill kernels: 32-bit scores, local, score and end cell only.
#include "dp_fill.h"

namespace mica {
void reg_fill_k32_1_0(KernelTable& t) {
  fill_bucket_table<kTbNone, kK32, 1>(t.bucket[0], ClassSeq{});
}
}  // namespace mica
