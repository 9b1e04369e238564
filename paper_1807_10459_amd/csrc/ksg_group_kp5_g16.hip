// Grouped search-kernel instantiations: 16 problems per group, 5 top-k registers
// (k <= 4), conditioning dimension m = 0..14.
#include "ksg_group.inc.h"

namespace ksg {

#define KSG_G(M) reinterpret_cast<const void*>(&ksg_group_kernel<M, 16, 5>)
const void* group_kernels_kp5_g16[15] = {KSG_G(0),  KSG_G(1),  KSG_G(2),  KSG_G(3), KSG_G(4),
                                        KSG_G(5),  KSG_G(6),  KSG_G(7),  KSG_G(8), KSG_G(9),
                                        KSG_G(10), KSG_G(11), KSG_G(12), KSG_G(13), KSG_G(14)};

}  // namespace ksg
