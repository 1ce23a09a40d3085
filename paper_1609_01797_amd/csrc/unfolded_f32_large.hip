// Unfolded TASER kernels in float, register buckets 56, 64.
#include "unfolded_kernels.h"

namespace taser {

template hipError_t unf_fwd<56, 1, float>(const UnfoldedArgs&, const void*, const void*,
                                           const void*, const void*, void*, void*, hipStream_t);
template hipError_t unf_bwd<56, 1, float>(const UnfoldedArgs&, const void*, const void*,
                                           const void*, const void*, const void*, const void*,
                                           void*, hipStream_t);
template hipError_t unf_fwd<64, 1, float>(const UnfoldedArgs&, const void*, const void*,
                                           const void*, const void*, void*, void*, hipStream_t);
template hipError_t unf_bwd<64, 1, float>(const UnfoldedArgs&, const void*, const void*,
                                           const void*, const void*, const void*, const void*,
                                           void*, hipStream_t);

}  // namespace taser
