// Persistent fill kernel: score and end cell only, seed extension, reads of 161-256 bases.
#include "dp_fill.h"

namespace mica {
void reg_persistent_0_2_1(KernelTable& t) { t.persistent[0][2][1] = &k_fill_persistent<kTbNone, 2, 1>; }
}  // namespace mica
