// Search-kernel instantiations for 17 top-k registers (k <= 16).
#include "ksg_search.inc.h"

namespace ksg {

#define KSG_ONE(S) reinterpret_cast<const void*>(&ksg_batch_kernel<S, 17>)
#define KSG_ROW(P)                                                                            \
  KSG_ONE((P) * 13 + 0), KSG_ONE((P) * 13 + 1), KSG_ONE((P) * 13 + 2), KSG_ONE((P) * 13 + 3), \
      KSG_ONE((P) * 13 + 4), KSG_ONE((P) * 13 + 5), KSG_ONE((P) * 13 + 6),                   \
      KSG_ONE((P) * 13 + 7), KSG_ONE((P) * 13 + 8), KSG_ONE((P) * 13 + 9),                   \
      KSG_ONE((P) * 13 + 10), KSG_ONE((P) * 13 + 11), KSG_ONE((P) * 13 + 12)

static_assert(kFastMaxDz + 1 == 13, "fast-shape table layout");

#define KSG_DIMS(D) KSG_ONE(kGenericShape + (D))

// [0, 39): single fast-shape kernels; [39]: mixed-shape kernel (per-problem dispatch);
// [40 + D - 2] for D in [2, 16]: kernels for generic shapes of D columns.
const void* search_kernels_kp17[55] = {
    KSG_ROW(0),   KSG_ROW(1),   KSG_ROW(2),   KSG_ONE(-1),  KSG_DIMS(2),  KSG_DIMS(3),
    KSG_DIMS(4),  KSG_DIMS(5),  KSG_DIMS(6),  KSG_DIMS(7),  KSG_DIMS(8),  KSG_DIMS(9),
    KSG_DIMS(10), KSG_DIMS(11), KSG_DIMS(12), KSG_DIMS(13), KSG_DIMS(14), KSG_DIMS(15),
    KSG_DIMS(16)};

}  // namespace ksg
