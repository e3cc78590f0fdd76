// Persistent fill kernel: score and end only, local.
#include "dp_fill.h"

namespace mica {
void reg_persistent_0_1(KernelTable& t) { t.persistent[0][1] = &k_fill_persistent<false, 1>; }
}  // namespace mica
