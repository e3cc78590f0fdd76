// Per-bucket fill kernels: packed 16-bit scores, local, with the banded traceback.
#include "dp_fill.h"

namespace mica {
void reg_fill_k16_1_1(KernelTable& t) {
  fill_bucket_table<kTbBand, kK16, 1>(t.bucket[1], ClassSeq{});
}
}  // namespace mica
