// Persistent fill kernel: score and end only, semi-global, reads of 161 to 256 bases.
#include "dp_fill.h"

namespace mica {
void reg_persistent_0_0_1(KernelTable& t) { t.persistent[0][0][1] = &k_fill_persistent<false, 0, 1>; }
}  // namespace mica
