// gather_c2_6.hip -- instances of the fused IFCM step for C = 2, 3, 5, 6.
#include "gather.h"

namespace pifcm {
PIFCM_DEFINE_GATHER(2, false)
PIFCM_DEFINE_GATHER(3, false)
PIFCM_DEFINE_GATHER(5, false)
PIFCM_DEFINE_GATHER(6, false)
}  // namespace pifcm
