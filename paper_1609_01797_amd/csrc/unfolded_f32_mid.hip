// Unfolded TASER kernels in float, register buckets 40, 48.
#include "unfolded_kernels.h"

namespace taser {

template hipError_t unf_fwd<40, 1, float>(const UnfoldedArgs&, const void*, const void*,
                                           const void*, const void*, void*, void*, hipStream_t);
template hipError_t unf_bwd<40, 1, float>(const UnfoldedArgs&, const void*, const void*,
                                           const void*, const void*, const void*, const void*,
                                           void*, hipStream_t);
template hipError_t unf_fwd<40, 2, float>(const UnfoldedArgs&, const void*, const void*,
                                           const void*, const void*, void*, void*, hipStream_t);
template hipError_t unf_bwd<40, 2, float>(const UnfoldedArgs&, const void*, const void*,
                                           const void*, const void*, const void*, const void*,
                                           void*, hipStream_t);
template hipError_t unf_fwd<48, 1, float>(const UnfoldedArgs&, const void*, const void*,
                                           const void*, const void*, void*, void*, hipStream_t);
template hipError_t unf_bwd<48, 1, float>(const UnfoldedArgs&, const void*, const void*,
                                           const void*, const void*, const void*, const void*,
                                           void*, hipStream_t);

}  // namespace taser
