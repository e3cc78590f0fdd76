// Full-traceback fill kernels for pairs whose band was too wide: packed 16-bit scores, local.
#include "dp_fill.h"

namespace mica {
void reg_fill_fb_k16_1(KernelTable& t) {
  fill_fallback_table<kK16, 1>(t.fallback, ClassSeq{});
}
}  // namespace mica
