// Persistent fill kernel: with the banded traceback, semi-global, reads of 161-256 bases.
#include "dp_fill.h"

namespace mica {
void reg_persistent_1_0_1(KernelTable& t) { t.persistent[1][0][1] = &k_fill_persistent<kTbBand, 0, 1>; }
}  // namespace mica
