// The LU panel leaf instantiated for two rows per thread (grids larger than
// the CU count), in a source of its own so that the two instantiations of
// the fully unrolled kernel compile in parallel.
#include "lu_leaf.h"

namespace cdf {

const void *leaf_kernel_r2() { return reinterpret_cast<const void *>(&lu_leaf_kernel<2>); }

}  // namespace cdf
