// Persistent fallback kernel: the full traceback of the wide-band pairs of the
// persistent buckets, seed extension, reads up to 160 bases.
#include "dp_fill.h"

namespace mica {
void reg_persistent_fb_2_0(KernelTable& t) { t.fb_persistent[2][0] = &k_fill_persistent<kTbFull, 2, 0, true>; }
}  // namespace mica
