// Key-ordered window search kernels for KSG algorithm 2 (neighbour rectangles), one per
// column count, top-k of 5 slots (k <= 4).
#include "ksg_window.inc.h"

namespace ksg {

#define KSG_WIN2(D) reinterpret_cast<const void*>(&ksg_window_kernel<D, 5, 2>)
// [D - 2] for D in [2, 16]
const void* window_kernels_alg2[15] = {KSG_WIN2(2),  KSG_WIN2(3),  KSG_WIN2(4),  KSG_WIN2(5),  KSG_WIN2(6),
                                       KSG_WIN2(7),  KSG_WIN2(8),  KSG_WIN2(9),  KSG_WIN2(10), KSG_WIN2(11),
                                       KSG_WIN2(12), KSG_WIN2(13), KSG_WIN2(14), KSG_WIN2(15), KSG_WIN2(16)};

}  // namespace ksg
