// Persistent band refill of the persistent buckets' pairs whose band has
// 17-64 diagonals, local, reads up to 160 bases.
#include "dp_fill.h"

namespace mica {
void reg_persistent_db_1_0(KernelTable& t) { t.db_persistent[1][0] = &k_fill_persistent<kTbDefer, 1, 0, true>; }
}  // namespace mica
