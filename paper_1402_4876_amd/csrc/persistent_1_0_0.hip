// Persistent fill kernel: with the banded traceback, semi-global, reads up to 160 bases.
#include "dp_fill.h"

namespace mica {
void reg_persistent_1_0_0(KernelTable& t) { t.persistent[1][0][0] = &k_fill_persistent<kTbBand, 0, 0>; }
}  // namespace mica
