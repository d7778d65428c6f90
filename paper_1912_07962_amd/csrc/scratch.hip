// Fixed device scratch of the allocation-free forward projection
// (slim_project_noalloc): the projector's partial sums for callers that
// cannot allocate device memory.  One array per device, loaded with the
// library's code object and held until the process ends.  In host code the
// symbol is only a stand-in; kernels receive the device address that
// hipGetSymbolAddress returns for the current device, kept per device.
#include "slim_internal.h"

#include <mutex>

namespace slim {

constexpr size_t kScratchFloats = size_t(4) << 20;  // 16 MiB
static __device__ __align__(256) float scratch[kScratchFloats];
constexpr int kMaxScratchDevices = 64;
static float* g_scratch[kMaxScratchDevices] = {};
static std::mutex g_scratch_mu;

size_t forward_scratch_floats() { return kScratchFloats; }

hipError_t forward_scratch_setup() {
  int dev = 0;
  hipError_t e = hipGetDevice(&dev);
  if (e != hipSuccess) return e;
  if (dev < 0 || dev >= kMaxScratchDevices) return hipErrorInvalidDevice;
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  if (g_scratch[dev]) return hipSuccess;
  void* p = nullptr;
  e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
  if (e != hipSuccess) return e;
  g_scratch[dev] = (float*)p;
  return hipSuccess;
}

float* forward_scratch(int dev) {
  if (dev < 0 || dev >= kMaxScratchDevices) return nullptr;
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  return g_scratch[dev];
}

}  // namespace slim
