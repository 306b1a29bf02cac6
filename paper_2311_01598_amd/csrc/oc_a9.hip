// oc_a9.hip -- Output-Centric kernels for a column pass of length 2^9.
#include "oc_kernels.h"

namespace ks {
template hipError_t oc_cols<9>(const Plan &, const OcArgs &, hipStream_t);
}  // namespace ks
