// Persistent band refill of the persistent buckets' pairs whose band has
// 17-64 diagonals, local, reads of 161-256 bases.
#include "dp_fill.h"

namespace mica {
void reg_persistent_db_1_1(KernelTable& t) { t.db_persistent[1][1] = &k_fill_persistent<kTbDefer, 1, 1, true>; }
}  // namespace mica
