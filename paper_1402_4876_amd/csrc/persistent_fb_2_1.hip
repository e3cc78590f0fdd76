// Persistent fallback kernel: the full traceback of the wide-band pairs of the
// persistent buckets, seed extension, reads of 161-256 bases.
#include "dp_fill.h"

namespace mica {
void reg_persistent_fb_2_1(KernelTable& t) { t.fb_persistent[2][1] = &k_fill_persistent<kTbFull, 2, 1, true>; }
}  // namespace mica
