// Persistent fill kernel: score and end cell only, semi-global, reads of 161-256 bases.
#include "dp_fill.h"

namespace mica {
void reg_persistent_0_0_1(KernelTable& t) { t.persistent[0][0][1] = &k_fill_persistent<kTbNone, 0, 1>; }
}  // namespace mica
