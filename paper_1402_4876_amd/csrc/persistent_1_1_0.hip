// Persistent fill kernel: with the banded traceback, local, reads up to 160 bases.
#include "dp_fill.h"

namespace mica {
void reg_persistent_1_1_0(KernelTable& t) { t.persistent[1][1][0] = &k_fill_persistent<kTbBand, 1, 0>; }
}  // namespace mica
