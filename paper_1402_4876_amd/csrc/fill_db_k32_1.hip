// Band refill of the pairs whose band has 17-64 diagonals: 32-bit scores, local.
#include "dp_fill.h"

namespace mica {
void reg_band_db_k32_1(KernelTable& t) {
  band_deferred_table<kK32, 1>(t.deferred, ClassSeq{});
}
}  // namespace mica
