// oc_a6.hip -- Output-Centric kernels for a column pass of length 2^6.
#include "oc_kernels.h"

namespace ks {
template hipError_t oc_cols<6>(const Plan &, const OcArgs &, hipStream_t);
}  // namespace ks
