// Persistent band refill of the persistent buckets' pairs whose band has
// 17-64 diagonals, extension, reads of 161-256 bases.
#include "dp_fill.h"

namespace mica {
void reg_persistent_db_2_1(KernelTable& t) { t.db_persistent[2][1] = &k_fill_persistent<kTbDefer, 2, 1, true>; }
}  // namespace mica
