// Hop kernel variants for FP32 storage.
#include "tm_hop.inc.h"

namespace twm {
TM_HOP_DEFINE(TM_FP32)
}  // namespace twm
