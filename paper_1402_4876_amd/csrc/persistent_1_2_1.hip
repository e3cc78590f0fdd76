// Persistent fill kernel: with the banded traceback, seed extension, reads of 161-256 bases.
#include "dp_fill.h"

namespace mica {
void reg_persistent_1_2_1(KernelTable& t) { t.persistent[1][2][1] = &k_fill_persistent<kTbBand, 2, 1>; }
}  // namespace mica
