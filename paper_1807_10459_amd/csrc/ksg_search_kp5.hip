// Search-kernel instantiations for 5 top-k registers (k <= 4).
#include "ksg_search.inc.h"

namespace ksg {

#define KSG_ONE(S) reinterpret_cast<const void*>(&ksg_batch_kernel<S, 5>)
#define KSG_ROW(P)                                                                            \
  KSG_ONE((P) * 13 + 0), KSG_ONE((P) * 13 + 1), KSG_ONE((P) * 13 + 2), KSG_ONE((P) * 13 + 3), \
      KSG_ONE((P) * 13 + 4), KSG_ONE((P) * 13 + 5), KSG_ONE((P) * 13 + 6),                   \
      KSG_ONE((P) * 13 + 7), KSG_ONE((P) * 13 + 8), KSG_ONE((P) * 13 + 9),                   \
      KSG_ONE((P) * 13 + 10), KSG_ONE((P) * 13 + 11), KSG_ONE((P) * 13 + 12)

static_assert(kFastMaxDz + 1 == 13, "fast-shape table layout");

// [0, 39): single-shape kernels; [39]: mixed-shape kernel (per-problem dispatch).
const void* search_kernels_kp5[40] = {KSG_ROW(0), KSG_ROW(1), KSG_ROW(2), KSG_ONE(-1)};

}  // namespace ksg
