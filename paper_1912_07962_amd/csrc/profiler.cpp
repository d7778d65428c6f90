// HIP-event timing of launch groups (see Profiler in slim_internal.h).
#include "slim_internal.h"

namespace slim {

hipError_t Profiler::begin(int k, hipStream_t st) {
  if ((size_t)(2 * used + 2) > pool.size()) {
    for (int q = 0; q < 64; ++q) {
      hipEvent_t ev;
      // no system-scope fence: the events time kernels on the device, and a
      // fence would add cache flushes inside the timed interval
      hipError_t e = hipEventCreateWithFlags(&ev, hipEventDisableSystemFence);
      if (e != hipSuccess) return e;
      pool.push_back(ev);
    }
  }
  if ((size_t)used >= kind.size()) kind.resize(used + 1);
  kind[used] = k;
  return hipEventRecord(pool[2 * used], st);
}

hipError_t Profiler::end(hipStream_t st) {
  hipError_t e = hipEventRecord(pool[2 * used + 1], st);
  ++used;
  return e;
}

hipError_t Profiler::harvest() {
  for (int q = 0; q < used; ++q) {
    float ms = 0.f;
    hipError_t e = hipEventElapsedTime(&ms, pool[2 * q], pool[2 * q + 1]);
    if (e != hipSuccess) return e;
    total_ms[kind[q]] += ms;
    launches[kind[q]] += 1;
  }
  used = 0;
  return hipSuccess;
}

void Profiler::release() {
  for (hipEvent_t ev : pool) (void)hipEventDestroy(ev);
  pool.clear();
  kind.clear();
  used = 0;
}

}  // namespace slim
