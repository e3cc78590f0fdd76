// Persistent band refill of the persistent buckets' pairs whose band has
// 17-64 diagonals, semi-global, reads of 161-256 bases.
#include "dp_fill.h"

namespace mica {
void reg_persistent_db_0_1(KernelTable& t) { t.db_persistent[0][1] = &k_fill_persistent<kTbDefer, 0, 1, true>; }
}  // namespace mica
