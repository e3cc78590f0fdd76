// Per-bucket fill kernels: packed 16-bit scores with a saturation check, local, score and end cell only.
#include "dp_fill.h"

namespace mica {
void reg_fill_k16s_1_0(KernelTable& t) {
  fill_bucket_table<kTbNone, kK16Sat, 1>(t.bucket[0], ClassSeq{});
}
}  // namespace mica
