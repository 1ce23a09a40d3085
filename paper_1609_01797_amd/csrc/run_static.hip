// Device-resident state for taser_run_static: the per-group state of the
// group path (G~, c~, D, tau and flags of each channel group, written by the
// preparation kernel and read by the solve kernel) in a file-scope device
// array, for callers that cannot allocate a workspace.
#include <mutex>

#include "taser_internal.h"

namespace taser {
namespace {

// 4,352 bytes of state per group of 16 vectors, for up to
// TASER_STATIC_MAX_VECTORS vectors: 17 MiB.  Every device the library runs
// on holds its own copy until the process ends.
constexpr size_t kScratchBytes = (size_t)(TASER_STATIC_MAX_VECTORS / 16) * kGroupWsBytes;
__device__ __align__(256) unsigned char scratch[kScratchBytes];

constexpr int kMaxDevices = 64;
std::mutex g_mu;
void* g_scratch[kMaxDevices];   // device address of `scratch`, per device

}  // namespace

size_t static_scratch_bytes() { return kScratchBytes; }

// The address of the current device's copy of `scratch`.  In host code the
// array's name is not a device address, so it is looked up once per device
// (with that device current) and kept; kernels get this pointer.
hipError_t static_scratch(void** ptr) {
  int dev = 0;
  hipError_t e = hipGetDevice(&dev);
  if (e != hipSuccess) return e;
  if (dev < 0 || dev >= kMaxDevices) return hipErrorInvalidDevice;
  std::lock_guard<std::mutex> lock(g_mu);
  if (!g_scratch[dev]) {
    void* p = nullptr;
    e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess) return e;
    g_scratch[dev] = p;
  }
  *ptr = g_scratch[dev];
  return hipSuccess;
}

}  // namespace taser
