// Persistent fill kernel (with traceback).
#include "dp_fill.h"

namespace mica {
void reg_persistent_1(KernelTable& t) { t.persistent[1] = &k_fill_persistent<true>; }
}  // namespace mica
