// Per-bucket fill kernels: 32-bit scores, local, with the banded traceback.
#include "dp_fill.h"

namespace mica {
void reg_fill_k32_1_1(KernelTable& t) {
  fill_bucket_table<kTbBand, kK32, 1>(t.bucket[1], ClassSeq{});
}
}  // namespace mica
