// Persistent fill kernel: score and end cell only, semi-global, reads up to 160 bases.
#include "dp_fill.h"

namespace mica {
void reg_persistent_0_0_0(KernelTable& t) { t.persistent[0][0][0] = &k_fill_persistent<kTbNone, 0, 0>; }
}  // namespace mica
