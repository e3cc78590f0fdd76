// Full-traceback fill kernels for pairs whose band was too wide: packed 16-bit scores with a saturation check, local.
#include "dp_fill.h"

namespace mica {
void reg_fill_fb_k16s_1(KernelTable& t) {
  fill_fallback_table<kK16Sat, 1>(t.fallback, ClassSeq{});
}
}  // namespace mica
