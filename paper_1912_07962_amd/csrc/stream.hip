// Streaming data (sec. 1: the rows of a block and their data are needed only
// when the block is sampled): a block's sinogram rows, delivered as one
// contiguous [B][n][R] array, are placed into the context's sinogram at
// their angle ids.
#include "slim_internal.h"

namespace slim {
namespace {

template <typename T>
__global__ __launch_bounds__(256) void scatter_rows_kernel(const T* __restrict__ in, int n_angles,
                                                           int R, AngleList ids,
                                                           T* __restrict__ b) {
  const int i = blockIdx.y, s = blockIdx.z;
  const int t = blockIdx.x * 256 + threadIdx.x;
  if (t >= R) return;
  b[((size_t)s * n_angles + ids.id[i]) * R + t] = in[((size_t)s * ids.n + i) * R + t];
}

}  // namespace

hipError_t launch_scatter_rows(const void* in, int bf16, int n_angles, int R, int B,
                               const AngleList& ids, void* b, hipStream_t st) {
  if (R < 1 || B < 1 || B > 65535 || ids.n < 1 || ids.n > 65535) return hipErrorInvalidValue;
  for (int i = 0; i < ids.n; ++i)
    if (ids.id[i] < 0 || ids.id[i] >= n_angles) return hipErrorInvalidValue;
  const dim3 grid((R + 255) / 256, ids.n, B);
  if (bf16)
    hipLaunchKernelGGL(scatter_rows_kernel<uint16_t>, grid, dim3(256), 0, st,
                       (const uint16_t*)in, n_angles, R, ids, (uint16_t*)b);
  else
    hipLaunchKernelGGL(scatter_rows_kernel<float>, grid, dim3(256), 0, st, (const float*)in,
                       n_angles, R, ids, (float*)b);
  return hipGetLastError();
}

}  // namespace slim
