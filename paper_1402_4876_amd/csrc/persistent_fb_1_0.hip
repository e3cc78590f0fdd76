// Persistent fallback kernel: the full traceback of the wide-band pairs of the
// persistent buckets, local, reads up to 160 bases.
#include "dp_fill.h"

namespace mica {
void reg_persistent_fb_1_0(KernelTable& t) { t.fb_persistent[1][0] = &k_fill_persistent<kTbFull, 1, 0, true>; }
}  // namespace mica
