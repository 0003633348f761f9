// Hop kernel variants for FP64 storage.
#include "tm_hop.inc.h"

namespace twm {
TM_HOP_DEFINE(TM_FP64)
}  // namespace twm
