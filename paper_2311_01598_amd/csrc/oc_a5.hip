// oc_a5.hip -- Output-Centric kernels for a column pass of length 2^5.
#include "oc_kernels.h"

namespace ks {
template hipError_t oc_cols<5>(const Plan &, const OcArgs &, hipStream_t);
}  // namespace ks
