// Full-traceback fill kernels for pairs whose band was too wide: packed 16-bit scores with a saturation check, semi-global.
#include "dp_fill.h"

namespace mica {
void reg_fill_fb_k16s_0(KernelTable& t) {
  fill_fallback_table<kK16Sat, 0>(t.fallback, ClassSeq{});
}
}  // namespace mica
