// oc_a4.hip -- Output-Centric kernels for a column pass of length 2^4.
#include "oc_kernels.h"

namespace ks {
template hipError_t oc_cols<4>(const Plan &, const OcArgs &, hipStream_t);
}  // namespace ks
