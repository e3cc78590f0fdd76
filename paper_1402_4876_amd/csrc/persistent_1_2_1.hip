// Persistent fill kernel: with traceback, extension, reads of 161 to 256 bases.
#include "dp_fill.h"

namespace mica {
void reg_persistent_1_2_1(KernelTable& t) { t.persistent[1][2][1] = &k_fill_persistent<true, 2, 1>; }
}  // namespace mica
