// Band refill of the pairs whose band has 17-64 diagonals: packed 16-bit scores, semi-global.
#include "dp_fill.h"

namespace mica {
void reg_band_db_k16_0(KernelTable& t) {
  band_deferred_table<kK16, 0>(t.deferred, ClassSeq{});
}
}  // namespace mica
