// Band refill of the pairs whose band has 17-64 diagonals: packed 16-bit scores with saturation checks, extension.
#include "dp_fill.h"

namespace mica {
void reg_band_db_k16s_2(KernelTable& t) {
  band_deferred_table<kK16Sat, 2>(t.deferred, ClassSeq{});
}
}  // namespace mica
