// Grouped search-kernel instantiations: 16 problems per group, 5 top-k registers
// (k <= 4), conditioning dimension m = 0..14.
#include "ksg_group.inc.h"

namespace ksg {

#define KSG_R(M) reinterpret_cast<const void*>(&ksg_group_radius_kernel<M, 16, 5>)
const void* group_radius_kernels_kp5_g16[15] = {KSG_R(0),  KSG_R(1),  KSG_R(2),  KSG_R(3),  KSG_R(4),
                                              KSG_R(5),  KSG_R(6),  KSG_R(7),  KSG_R(8),  KSG_R(9),
                                              KSG_R(10), KSG_R(11), KSG_R(12), KSG_R(13), KSG_R(14)};

// The X count kernels do not depend on k; they are instantiated once per group size.
#define KSG_X(M) reinterpret_cast<const void*>(&ksg_group_xcount_kernel<M, 16>)
const void* group_xcount_kernels_g16[15] = {KSG_X(0),  KSG_X(1),  KSG_X(2),  KSG_X(3),  KSG_X(4),
                                             KSG_X(5),  KSG_X(6),  KSG_X(7),  KSG_X(8),  KSG_X(9),
                                             KSG_X(10), KSG_X(11), KSG_X(12), KSG_X(13), KSG_X(14)};

}  // namespace ksg
