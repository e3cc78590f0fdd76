// Side lists after the banded fill of each bucket (full traceback of the
// pairs whose band was too wide, band refill of bands of 17-64 diagonals):
// 32-bit scores, local.
#include "dp_fill.h"

namespace mica {
void reg_side_k32_1(KernelTable& t) {
  side_bucket_table<kK32, 1>(t.side, ClassSeq{});
}
}  // namespace mica
