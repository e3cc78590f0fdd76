// Band refill of the pairs whose band has 17-64 diagonals: 32-bit scores, semi-global.
#include "dp_fill.h"

namespace mica {
void reg_band_db_k32_0(KernelTable& t) {
  band_deferred_table<kK32, 0>(t.deferred, ClassSeq{});
}
}  // namespace mica
