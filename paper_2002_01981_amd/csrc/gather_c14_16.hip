// gather_c14_16.hip -- instances of the fused IFCM step for C = 14, 15, 16.
#include "gather.h"

namespace pifcm {
PIFCM_DEFINE_GATHER(14, false)
PIFCM_DEFINE_GATHER(15, false)
PIFCM_DEFINE_GATHER(16, false)
}  // namespace pifcm
