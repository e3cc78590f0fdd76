// Persistent fill kernel: score and end cell only, seed extension, reads up to 160 bases.
#include "dp_fill.h"

namespace mica {
void reg_persistent_0_2_0(KernelTable& t) { t.persistent[0][2][0] = &k_fill_persistent<kTbNone, 2, 0>; }
}  // namespace mica
