// gather_c11_13.hip -- instances of the fused IFCM step for C = 11, 12, 13.
#include "gather.h"

namespace pifcm {
PIFCM_DEFINE_GATHER(11, false)
PIFCM_DEFINE_GATHER(12, false)
PIFCM_DEFINE_GATHER(13, false)
}  // namespace pifcm
