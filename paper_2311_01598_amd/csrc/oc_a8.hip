// oc_a8.hip -- Output-Centric kernels for a column pass of length 2^8.
#include "oc_kernels.h"

namespace ks {
template hipError_t oc_cols<8>(const Plan &, const OcArgs &, hipStream_t);
}  // namespace ks
