// Persistent band refill of the persistent buckets' pairs whose band has
// 17-64 diagonals, extension, reads up to 160 bases.
#include "dp_fill.h"

namespace mica {
void reg_persistent_db_2_0(KernelTable& t) { t.db_persistent[2][0] = &k_fill_persistent<kTbDefer, 2, 0, true>; }
}  // namespace mica
