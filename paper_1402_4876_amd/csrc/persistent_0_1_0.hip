// Persistent fill kernel: score and end cell only, local, reads up to 160 bases.
#include "dp_fill.h"

namespace mica {
void reg_persistent_0_1_0(KernelTable& t) { t.persistent[0][1][0] = &k_fill_persistent<kTbNone, 1, 0>; }
}  // namespace mica
