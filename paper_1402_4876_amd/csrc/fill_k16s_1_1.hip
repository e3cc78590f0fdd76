// Per-bucket fill kernels: packed 16-bit scores with saturation check, local, with traceback.
#include "dp_fill.h"

namespace mica {
void reg_fill_k16s_1_1(KernelTable& t) {
  fill_bucket_table<true, kK16Sat, 1>(t.bucket[1], ClassSeq{});
}
}  // namespace mica
