// Grouped search-kernel instantiations for conditioning dimensions m = 15..30: 8 problems per
// group, 9 top-k registers (k <= 8).
#include "ksg_group.inc.h"

namespace ksg {

#define KSG_R(M) reinterpret_cast<const void*>(&ksg_group_radius_kernel<M, 8, 9>)
const void* group_radius_kernels_kp9_g8_wide[16] = {
    KSG_R(15), KSG_R(16), KSG_R(17), KSG_R(18), KSG_R(19), KSG_R(20), KSG_R(21), KSG_R(22),
    KSG_R(23), KSG_R(24), KSG_R(25), KSG_R(26), KSG_R(27), KSG_R(28), KSG_R(29), KSG_R(30)};

}  // namespace ksg
