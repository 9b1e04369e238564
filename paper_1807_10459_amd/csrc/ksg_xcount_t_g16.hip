// Transposed X count kernel instantiations, 16 problems per group, conditioning dimension m = 0..14.
#include "ksg_xcount_t.inc.h"

namespace ksg {

#define KSG_XT(M) reinterpret_cast<const void*>(&ksg_group_xcount_t_kernel<M, 16>)
const void* group_xcount_t_kernels_g16[kGroupMaxM16 + 1] = {
    KSG_XT(0), KSG_XT(1), KSG_XT(2),  KSG_XT(3),  KSG_XT(4),  KSG_XT(5),  KSG_XT(6), KSG_XT(7),
    KSG_XT(8), KSG_XT(9), KSG_XT(10), KSG_XT(11), KSG_XT(12), KSG_XT(13), KSG_XT(14)};
static_assert(kGroupMaxM16 == 14, "one instantiation per conditioning dimension");

}  // namespace ksg
