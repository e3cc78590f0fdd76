// Full-traceback fill kernels for pairs whose band was too wide: 32-bit scores, semi-global.
#include "dp_fill.h"

namespace mica {
void reg_fill_fb_k32_0(KernelTable& t) {
  fill_fallback_table<kK32, 0>(t.fallback, ClassSeq{});
}
}  // namespace mica
