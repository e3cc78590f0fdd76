// Persistent kernel over the side lists of the persistent buckets (full
// traceback of the pairs whose band was too wide, then band refill of bands
// of 17-64 diagonals), semi-global, reads of 161-256 bases.
#include "dp_fill.h"

namespace mica {
void reg_persistent_side_0_1(KernelTable& t) { t.side_persistent[0][1] = &k_side_persistent<0, 1>; }
}  // namespace mica
