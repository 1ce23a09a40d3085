// Unfolded TASER kernels in double, register buckets 8, 16, 24, 32.
#include "unfolded_kernels.h"

namespace taser {

template hipError_t unf_fwd<8, 1, double>(const UnfoldedArgs&, const void*, const void*,
                                           const void*, const void*, void*, void*, hipStream_t);
template hipError_t unf_bwd<8, 1, double>(const UnfoldedArgs&, const void*, const void*,
                                           const void*, const void*, const void*, const void*,
                                           void*, hipStream_t);
template hipError_t unf_fwd<16, 1, double>(const UnfoldedArgs&, const void*, const void*,
                                           const void*, const void*, void*, void*, hipStream_t);
template hipError_t unf_bwd<16, 1, double>(const UnfoldedArgs&, const void*, const void*,
                                           const void*, const void*, const void*, const void*,
                                           void*, hipStream_t);
template hipError_t unf_fwd<24, 1, double>(const UnfoldedArgs&, const void*, const void*,
                                           const void*, const void*, void*, void*, hipStream_t);
template hipError_t unf_bwd<24, 1, double>(const UnfoldedArgs&, const void*, const void*,
                                           const void*, const void*, const void*, const void*,
                                           void*, hipStream_t);
template hipError_t unf_fwd<32, 1, double>(const UnfoldedArgs&, const void*, const void*,
                                           const void*, const void*, void*, void*, hipStream_t);
template hipError_t unf_bwd<32, 1, double>(const UnfoldedArgs&, const void*, const void*,
                                           const void*, const void*, const void*, const void*,
                                           void*, hipStream_t);

}  // namespace taser
