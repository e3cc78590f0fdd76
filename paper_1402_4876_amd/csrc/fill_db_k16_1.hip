// Band refill of the pairs whose band has 17-64 diagonals: packed 16-bit scores, local.
#include "dp_fill.h"

namespace mica {
void reg_band_db_k16_1(KernelTable& t) {
  band_deferred_table<kK16, 1>(t.deferred, ClassSeq{});
}
}  // namespace mica
