// Unfolded TASER kernels in float, register buckets 8, 16, 24, 32.
#include "unfolded_kernels.h"

namespace taser {

template hipError_t unf_fwd<8, float>(const UnfoldedArgs&, const void*, const void*,
                                        const void*, const void*, void*, void*, hipStream_t);
template hipError_t unf_bwd<8, float>(const UnfoldedArgs&, const void*, const void*,
                                        const void*, const void*, const void*, const void*,
                                        void*, hipStream_t);
template hipError_t unf_fwd<16, float>(const UnfoldedArgs&, const void*, const void*,
                                        const void*, const void*, void*, void*, hipStream_t);
template hipError_t unf_bwd<16, float>(const UnfoldedArgs&, const void*, const void*,
                                        const void*, const void*, const void*, const void*,
                                        void*, hipStream_t);
template hipError_t unf_fwd<24, float>(const UnfoldedArgs&, const void*, const void*,
                                        const void*, const void*, void*, void*, hipStream_t);
template hipError_t unf_bwd<24, float>(const UnfoldedArgs&, const void*, const void*,
                                        const void*, const void*, const void*, const void*,
                                        void*, hipStream_t);
template hipError_t unf_fwd<32, float>(const UnfoldedArgs&, const void*, const void*,
                                        const void*, const void*, void*, void*, hipStream_t);
template hipError_t unf_bwd<32, float>(const UnfoldedArgs&, const void*, const void*,
                                        const void*, const void*, const void*, const void*,
                                        void*, hipStream_t);

}  // namespace taser
