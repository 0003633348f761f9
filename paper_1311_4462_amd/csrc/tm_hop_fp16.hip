// Hop kernel variants for FP16 storage.
#include "tm_hop.inc.h"

namespace twm {
TM_HOP_DEFINE(TM_FP16)
}  // namespace twm
