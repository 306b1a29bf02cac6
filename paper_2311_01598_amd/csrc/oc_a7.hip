// oc_a7.hip -- Output-Centric kernels for a column pass of length 2^7.
#include "oc_kernels.h"

namespace ks {
template hipError_t oc_cols<7>(const Plan &, const OcArgs &, hipStream_t);
}  // namespace ks
