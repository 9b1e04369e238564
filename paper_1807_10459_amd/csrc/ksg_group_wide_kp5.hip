// Grouped search-kernel instantiations for conditioning dimensions m = 15..30: 8 problems per
// group, 5 top-k registers (k <= 4); the X count kernels of the same m.
#include "ksg_group.inc.h"

namespace ksg {

#define KSG_R(M) reinterpret_cast<const void*>(&ksg_group_radius_kernel<M, 8, 5>)
const void* group_radius_kernels_kp5_g8_wide[16] = {
    KSG_R(15), KSG_R(16), KSG_R(17), KSG_R(18), KSG_R(19), KSG_R(20), KSG_R(21), KSG_R(22),
    KSG_R(23), KSG_R(24), KSG_R(25), KSG_R(26), KSG_R(27), KSG_R(28), KSG_R(29), KSG_R(30)};

#define KSG_X(M) reinterpret_cast<const void*>(&ksg_group_xcount_kernel<M, 8>)
const void* group_xcount_kernels_g8_wide[16] = {
    KSG_X(15), KSG_X(16), KSG_X(17), KSG_X(18), KSG_X(19), KSG_X(20), KSG_X(21), KSG_X(22),
    KSG_X(23), KSG_X(24), KSG_X(25), KSG_X(26), KSG_X(27), KSG_X(28), KSG_X(29), KSG_X(30)};

static_assert(kGroupMaxM == 30, "one instantiation per conditioning dimension 15..kGroupMaxM");

}  // namespace ksg
