// Per-bucket fill kernels: packed 16-bit scores, seed extension, score and end cell only.
#include "dp_fill.h"

namespace mica {
void reg_fill_k16_2_0(KernelTable& t) {
  fill_bucket_table<kTbNone, kK16, 2>(t.bucket[0], ClassSeq{});
}
}  // namespace mica
