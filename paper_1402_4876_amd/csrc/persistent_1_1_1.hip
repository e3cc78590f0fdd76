// Persistent fill kernel: with the banded traceback, local, reads of 161-256 bases.
#include "dp_fill.h"

namespace mica {
void reg_persistent_1_1_1(KernelTable& t) { t.persistent[1][1][1] = &k_fill_persistent<kTbBand, 1, 1>; }
}  // namespace mica
