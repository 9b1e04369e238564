// Grouped search-kernel instantiations: 8 problems per group, 9 top-k registers
// (k <= 8), conditioning dimension m = 0..14.
#include "ksg_group.inc.h"

namespace ksg {

#define KSG_R(M) reinterpret_cast<const void*>(&ksg_group_radius_kernel<M, 8, 9>)
const void* group_radius_kernels_kp9_g8[15] = {KSG_R(0),  KSG_R(1),  KSG_R(2),  KSG_R(3),  KSG_R(4),
                                              KSG_R(5),  KSG_R(6),  KSG_R(7),  KSG_R(8),  KSG_R(9),
                                              KSG_R(10), KSG_R(11), KSG_R(12), KSG_R(13), KSG_R(14)};

}  // namespace ksg
