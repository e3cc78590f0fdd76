// Persistent fill kernel: score and end only, extension, reads of 161 to 256 bases.
#include "dp_fill.h"

namespace mica {
void reg_persistent_0_2_1(KernelTable& t) { t.persistent[0][2][1] = &k_fill_persistent<false, 2, 1>; }
}  // namespace mica
