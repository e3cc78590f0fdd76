// Full-traceback fill kernels for pairs whose band was too wide: 32-bit scores, seed extension.
#include "dp_fill.h"

namespace mica {
void reg_fill_fb_k32_2(KernelTable& t) {
  fill_fallback_table<kK32, 2>(t.fallback, ClassSeq{});
}
}  // namespace mica
