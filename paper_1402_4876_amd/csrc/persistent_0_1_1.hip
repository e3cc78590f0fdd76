// Persistent fill kernel: score and end cell only, local, reads of 161-256 bases.
#include "dp_fill.h"

namespace mica {
void reg_persistent_0_1_1(KernelTable& t) { t.persistent[0][1][1] = &k_fill_persistent<kTbNone, 1, 1>; }
}  // namespace mica
