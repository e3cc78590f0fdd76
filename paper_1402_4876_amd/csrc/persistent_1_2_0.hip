// Persistent fill kernel: with the banded traceback, seed extension, reads up to 160 bases.
#include "dp_fill.h"

namespace mica {
void reg_persistent_1_2_0(KernelTable& t) { t.persistent[1][2][0] = &k_fill_persistent<kTbBand, 2, 0>; }
}  // namespace mica
