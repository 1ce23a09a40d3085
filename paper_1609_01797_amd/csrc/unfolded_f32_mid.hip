// Unfolded TASER kernels in float, register buckets 40, 48.
#include "unfolded_kernels.h"

namespace taser {

template hipError_t unf_fwd<40, float>(const UnfoldedArgs&, const void*, const void*,
                                        const void*, const void*, void*, void*, hipStream_t);
template hipError_t unf_bwd<40, float>(const UnfoldedArgs&, const void*, const void*,
                                        const void*, const void*, const void*, const void*,
                                        void*, hipStream_t);
template hipError_t unf_fwd<48, float>(const UnfoldedArgs&, const void*, const void*,
                                        const void*, const void*, void*, void*, hipStream_t);
template hipError_t unf_bwd<48, float>(const UnfoldedArgs&, const void*, const void*,
                                        const void*, const void*, const void*, const void*,
                                        void*, hipStream_t);

}  // namespace taser
