// gather_c4.hip -- instances of the fused IFCM step for C = 4.
#include "gather.h"

namespace pifcm {
PIFCM_DEFINE_GATHER(4, true)
}  // namespace pifcm
