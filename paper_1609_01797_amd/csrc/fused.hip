// Fused single-launch TASER (placeholder until the MFMA kernel lands).
#include "taser_internal.h"

namespace taser {

bool fused_supported(const FusedArgs&) { return false; }

hipError_t launch_fused(const FusedArgs&, hipStream_t) { return hipErrorNotSupported; }

}  // namespace taser
