// oc_a7.hip -- Output-Centric kernels for a column pass of length 2^7.
#include "oc_persist.h"

namespace ks {
template hipError_t oc_phases<7>(const Plan &, const OcJob &, const OcJob *, uint32_t, const uint32_t *, uint32_t,
                                  OcRowVariant, OcPart, hipStream_t);
template hipError_t oc_persistent<7>(const Plan &, const OcJob *, const OcSeg *, uint32_t, uint32_t, uint32_t,
                                      uint32_t *, uint32_t, hipStream_t);
}  // namespace ks
