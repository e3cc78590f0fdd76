// Side lists after the banded fill of each bucket (full traceback of the
// pairs whose band was too wide, band refill of bands of 17-64 diagonals):
// packed 16-bit scores with saturation checks, semi-global.
#include "dp_fill.h"

namespace mica {
void reg_side_k16s_0(KernelTable& t) {
  side_bucket_table<kK16Sat, 0>(t.side, ClassSeq{});
}
}  // namespace mica
