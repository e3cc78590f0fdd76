// Persistent fill kernel (score and end only).
#include "dp_fill.h"

namespace mica {
void reg_persistent_0(KernelTable& t) { t.persistent[0] = &k_fill_persistent<false>; }
}  // namespace mica
