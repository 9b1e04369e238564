// Transposed X count kernel instantiations, 8 problems per group, conditioning dimension m = 0..30.
#include "ksg_xcount_t.inc.h"

namespace ksg {

#define KSG_XT(M) reinterpret_cast<const void*>(&ksg_group_xcount_t_kernel<M, 8>)
const void* group_xcount_t_kernels_g8[kGroupMaxM + 1] = {
    KSG_XT(0),  KSG_XT(1),  KSG_XT(2),  KSG_XT(3),  KSG_XT(4),  KSG_XT(5),  KSG_XT(6),  KSG_XT(7),
    KSG_XT(8),  KSG_XT(9),  KSG_XT(10), KSG_XT(11), KSG_XT(12), KSG_XT(13), KSG_XT(14), KSG_XT(15),
    KSG_XT(16), KSG_XT(17), KSG_XT(18), KSG_XT(19), KSG_XT(20), KSG_XT(21), KSG_XT(22), KSG_XT(23),
    KSG_XT(24), KSG_XT(25), KSG_XT(26), KSG_XT(27), KSG_XT(28), KSG_XT(29), KSG_XT(30)};
static_assert(kGroupMaxM == 30, "one instantiation per conditioning dimension");

}  // namespace ksg
