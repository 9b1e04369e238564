// Search-kernel instantiations for problems of 17..32 columns: every such problem is searched
// as a problem of kWideDims columns whose Z is filled up with zero columns (zero in the N rows,
// +inf in the padding rows like every column).  A zero column adds |0 - 0| = 0 to a maximum of
// non-negative distances, so every radius and every count is that of the problem without it;
// with no real Z column, d^Z is 0 for every pair of real rows and n_Z comes out as N - 1
// (eps > 0) or 0 (eps = 0), the values the estimator takes for an empty Z.
#include "ksg_search.inc.h"

namespace ksg {

static_assert(kWideDims == kMaxDims, "wide problems fill up to the library's column limit");

// [0]: 5 top-k slots (k <= 4), [1]: 9 (k <= 8), [2]: 17 (k <= 16).
const void* search_kernels_wide[3] = {
    reinterpret_cast<const void*>(&ksg_batch_kernel<kGenericShape + kWideDims, 5>),
    reinterpret_cast<const void*>(&ksg_batch_kernel<kGenericShape + kWideDims, 9>),
    reinterpret_cast<const void*>(&ksg_batch_kernel<kGenericShape + kWideDims, 17>)};

}  // namespace ksg
