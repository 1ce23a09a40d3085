// Unfolded TASER kernels in float, register buckets 8, 16, 24, 32.
#include "unfolded_kernels.h"

namespace taser {

template hipError_t unf_fwd<8, 1, float>(const UnfoldedArgs&, const void*, const void*,
                                           const void*, const void*, void*, void*, hipStream_t);
template hipError_t unf_bwd<8, 1, float>(const UnfoldedArgs&, const void*, const void*,
                                           const void*, const void*, const void*, const void*,
                                           void*, hipStream_t);
template hipError_t unf_fwd<8, 2, float>(const UnfoldedArgs&, const void*, const void*,
                                           const void*, const void*, void*, void*, hipStream_t);
template hipError_t unf_bwd<8, 2, float>(const UnfoldedArgs&, const void*, const void*,
                                           const void*, const void*, const void*, const void*,
                                           void*, hipStream_t);
template hipError_t unf_fwd<16, 1, float>(const UnfoldedArgs&, const void*, const void*,
                                           const void*, const void*, void*, void*, hipStream_t);
template hipError_t unf_bwd<16, 1, float>(const UnfoldedArgs&, const void*, const void*,
                                           const void*, const void*, const void*, const void*,
                                           void*, hipStream_t);
template hipError_t unf_fwd<16, 2, float>(const UnfoldedArgs&, const void*, const void*,
                                           const void*, const void*, void*, void*, hipStream_t);
template hipError_t unf_bwd<16, 2, float>(const UnfoldedArgs&, const void*, const void*,
                                           const void*, const void*, const void*, const void*,
                                           void*, hipStream_t);
template hipError_t unf_fwd<24, 1, float>(const UnfoldedArgs&, const void*, const void*,
                                           const void*, const void*, void*, void*, hipStream_t);
template hipError_t unf_bwd<24, 1, float>(const UnfoldedArgs&, const void*, const void*,
                                           const void*, const void*, const void*, const void*,
                                           void*, hipStream_t);
template hipError_t unf_fwd<24, 2, float>(const UnfoldedArgs&, const void*, const void*,
                                           const void*, const void*, void*, void*, hipStream_t);
template hipError_t unf_bwd<24, 2, float>(const UnfoldedArgs&, const void*, const void*,
                                           const void*, const void*, const void*, const void*,
                                           void*, hipStream_t);
template hipError_t unf_fwd<32, 1, float>(const UnfoldedArgs&, const void*, const void*,
                                           const void*, const void*, void*, void*, hipStream_t);
template hipError_t unf_bwd<32, 1, float>(const UnfoldedArgs&, const void*, const void*,
                                           const void*, const void*, const void*, const void*,
                                           void*, hipStream_t);
template hipError_t unf_fwd<32, 2, float>(const UnfoldedArgs&, const void*, const void*,
                                           const void*, const void*, void*, void*, hipStream_t);
template hipError_t unf_bwd<32, 2, float>(const UnfoldedArgs&, const void*, const void*,
                                           const void*, const void*, const void*, const void*,
                                           void*, hipStream_t);

}  // namespace taser
