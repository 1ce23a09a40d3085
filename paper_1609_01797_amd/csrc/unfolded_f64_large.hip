// Unfolded TASER kernels in double, register buckets 56, 64.
#include "unfolded_kernels.h"

namespace taser {

template hipError_t unf_fwd<56, 1, double>(const UnfoldedArgs&, const void*, const void*,
                                           const void*, const void*, void*, void*, hipStream_t);
template hipError_t unf_bwd<56, 1, double>(const UnfoldedArgs&, const void*, const void*,
                                           const void*, const void*, const void*, const void*,
                                           void*, hipStream_t);
template hipError_t unf_fwd<64, 1, double>(const UnfoldedArgs&, const void*, const void*,
                                           const void*, const void*, void*, void*, hipStream_t);
template hipError_t unf_bwd<64, 1, double>(const UnfoldedArgs&, const void*, const void*,
                                           const void*, const void*, const void*, const void*,
                                           void*, hipStream_t);

}  // namespace taser
