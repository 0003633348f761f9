// Hop kernel variants for BF16 storage.
#include "tm_hop.inc.h"

namespace twm {
TM_HOP_DEFINE(TM_BF16)
}  // namespace twm
