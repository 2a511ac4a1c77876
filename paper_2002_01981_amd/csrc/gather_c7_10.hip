// gather_c7_10.hip -- instances of the fused IFCM step for C = 7, 8, 9, 10.
#include "gather.h"

namespace pifcm {
PIFCM_DEFINE_GATHER(7, false)
PIFCM_DEFINE_GATHER(8, false)
PIFCM_DEFINE_GATHER(9, false)
PIFCM_DEFINE_GATHER(10, false)
}  // namespace pifcm
