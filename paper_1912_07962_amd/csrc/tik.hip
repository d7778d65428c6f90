// Right-hand side of the slimTik step (sec. 2, eq. (slimTik)) with L = I in
// the Gram form: with mu = 1/alpha_k + W tik^2 / M and c = (tik^2 / M) / mu,
//   (M M^T + mu I) z = [0; ...; 0; res] - c M x,   s = M^T z + c x.
#include "slim_internal.h"

namespace slim {
namespace {

__global__ __launch_bounds__(256) void tik_rhs_kernel(const double* __restrict__ mx,
                                                      size_t mx_stride,
                                                      const double* __restrict__ res,
                                                      size_t res_stride, int p, int nres, double c,
                                                      double* __restrict__ rhs,
                                                      size_t rhs_stride) {
  const int j = blockIdx.x * 256 + threadIdx.x;
  const int sl = blockIdx.y;
  if (j >= p) return;
  double v = -c * mx[(size_t)sl * mx_stride + j];
  if (j >= p - nres) v += res[(size_t)sl * res_stride + j - (p - nres)];
  rhs[(size_t)sl * rhs_stride + j] = v;
}

}  // namespace

hipError_t launch_tik_rhs(const double* mx, size_t mx_stride, const double* res,
                          size_t res_stride, int p, int nres, double c, double* rhs,
                          size_t rhs_stride, int B, hipStream_t st) {
  if (p <= 0 || nres < 0 || nres > p || B < 1 || B > 65535) return hipErrorInvalidValue;
  hipLaunchKernelGGL(tik_rhs_kernel, dim3((p + 255) / 256, B), dim3(256), 0, st, mx, mx_stride,
                     res, res_stride, p, nres, c, rhs, rhs_stride);
  return hipGetLastError();
}

}  // namespace slim
