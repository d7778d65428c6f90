// FP64 Cholesky of the Gram system (lambda I + M M^T) and its triangular
// solves, for the explicit-Gram mode (p up to a few thousand).
//
// Blocked right-looking factorisation, panel width 64, row-major lower
// triangle: per panel one workgroup factors the diagonal block in LDS,
// a row-parallel kernel solves the panel below it against L11^T, and a
// tiled kernel applies the symmetric rank-64 update to the trailing lower
// triangle with float64 MFMA (v_mfma_f64_16x16x4f64).
//
// The right-hand side [0; ...; 0; res] is zero outside the newest block, so
// the forward solve only touches the trailing nr x nr triangle; the backward
// solve covers all p rows.  Both run in one workgroup with the vector in LDS.
#include "slim_internal.h"

namespace slim {

namespace {

constexpr int kNB = 64;

__global__ __launch_bounds__(256) void potrf_diag_kernel(double* __restrict__ G, int64_t ld, int k0,
                                                         int nb, int* __restrict__ info) {
  __shared__ double A[kNB][kNB + 1];
  for (int e = threadIdx.x; e < nb * nb; e += 256) {
    const int r = e / nb, c = e % nb;
    A[r][c] = (c <= r) ? G[(int64_t)(k0 + r) * ld + (k0 + c)] : 0.0;
  }
  __syncthreads();
  for (int j = 0; j < nb; ++j) {
    __shared__ double piv;
    if (threadIdx.x == 0) {
      double d = A[j][j];
      if (!(d > 0.0)) {  // catches NaN too
        if (info) atomicCAS(info, 0, k0 + j + 1);
        d = 1.0;
      }
      piv = sqrt(d);
      A[j][j] = piv;
    }
    __syncthreads();
    for (int i = j + 1 + threadIdx.x; i < nb; i += 256) A[i][j] /= piv;
    __syncthreads();
    for (int e = threadIdx.x; e < (nb - j - 1) * (nb - j - 1); e += 256) {
      const int i = j + 1 + e / (nb - j - 1);
      const int k = j + 1 + e % (nb - j - 1);
      if (k <= i) A[i][k] -= A[i][j] * A[k][j];
    }
    __syncthreads();
  }
  for (int e = threadIdx.x; e < nb * nb; e += 256) {
    const int r = e / nb, c = e % nb;
    if (c <= r) G[(int64_t)(k0 + r) * ld + (k0 + c)] = A[r][c];
  }
}

// rows i in [k0+nb, p): L21[i, :] = A21[i, :] L11^{-T}
__global__ __launch_bounds__(256) void trsm_panel_kernel(double* __restrict__ G, int64_t ld, int k0,
                                                         int nb, int p) {
  __shared__ double L[kNB][kNB + 1];
  for (int e = threadIdx.x; e < nb * nb; e += 256) {
    const int r = e / nb, c = e % nb;
    L[r][c] = (c <= r) ? G[(int64_t)(k0 + r) * ld + (k0 + c)] : 0.0;
  }
  __syncthreads();
  const int i = k0 + nb + blockIdx.x * 256 + threadIdx.x;
  if (i >= p) return;
  double x[kNB];
  double* row = G + (int64_t)i * ld + k0;
#pragma unroll
  for (int j = 0; j < kNB; ++j) x[j] = (j < nb) ? row[j] : 0.0;
#pragma unroll
  for (int j = 0; j < kNB; ++j) {
    if (j < nb) {
      double v = x[j];
#pragma unroll
      for (int q = 0; q < kNB; ++q)
        if (q < j) v -= x[q] * L[j][q];
      x[j] = v / L[j][j];
    }
  }
#pragma unroll
  for (int j = 0; j < kNB; ++j)
    if (j < nb) row[j] = x[j];
}

// Trailing update A22 -= L21 L21^T on 64x64 lower tiles, K = nb <= 64.
// 4 wavefronts; wavefront w computes the 16-row strip w of the tile as four
// 16x16 MFMA blocks.
typedef double double4_t __attribute__((ext_vector_type(4)));

__global__ __launch_bounds__(256) void syrk_update_kernel(double* __restrict__ G, int64_t ld, int k0,
                                                          int nb, int p) {
  const int ti = blockIdx.y, tj = blockIdx.x;
  if (tj > ti) return;
  const int base = k0 + nb;
  const int r0 = base + ti * 64, c0 = base + tj * 64;
  __shared__ double Li[64][kNB + 1];
  __shared__ double Lj[64][kNB + 1];
  for (int e = threadIdx.x; e < 64 * kNB; e += 256) {
    const int r = e / kNB, q = e % kNB;
    const bool okq = q < nb;
    Li[r][q] = (okq && r0 + r < p) ? G[(int64_t)(r0 + r) * ld + k0 + q] : 0.0;
    Lj[r][q] = (okq && c0 + r < p) ? G[(int64_t)(c0 + r) * ld + k0 + q] : 0.0;
  }
  __syncthreads();
  const int w = threadIdx.x >> 6;
  const int lane = threadIdx.x & 63;
  // v_mfma_f64_16x16x4f64: A is 16x4 (lane l holds A[l%16][l/16]), B is 4x16
  // (lane l holds B[l/16][l%16]); D is 16x16 and accumulator v of lane l
  // holds D[4*v + l/16][l%16] (rows interleaved across the accumulators).
  double4_t acc[4];
#pragma unroll
  for (int cb = 0; cb < 4; ++cb) acc[cb] = (double4_t){0.0, 0.0, 0.0, 0.0};
  const int ar = w * 16 + (lane & 15);
  const int kq = lane >> 4;
  for (int k = 0; k < kNB; k += 4) {
    const double av = Li[ar][k + kq];
#pragma unroll
    for (int cb = 0; cb < 4; ++cb) {
      const double bv = Lj[cb * 16 + (lane & 15)][k + kq];
      acc[cb] = __builtin_amdgcn_mfma_f64_16x16x4f64(av, bv, acc[cb], 0, 0, 0);
    }
  }
#pragma unroll
  for (int cb = 0; cb < 4; ++cb) {
#pragma unroll
    for (int v = 0; v < 4; ++v) {
      const int r = r0 + w * 16 + 4 * v + (lane >> 4);
      const int c = c0 + cb * 16 + (lane & 15);
      if (r < p && c < p && c <= r) G[(int64_t)r * ld + c] -= acc[cb][v];
    }
  }
}

// Triangular solves, one workgroup per right-hand side, vector in LDS.
constexpr int kSolveMax = 12288;

__global__ __launch_bounds__(1024) void chol_solve_kernel(const double* __restrict__ L, int64_t ld,
                                                          int p, int nr,
                                                          const double* __restrict__ rhs_all,
                                                          size_t rhs_stride,
                                                          double* __restrict__ z_all,
                                                          size_t z_stride) {
  extern __shared__ double y[];
  const double* rhs = rhs_all + (size_t)blockIdx.x * rhs_stride;
  double* z = z_all + (size_t)blockIdx.x * z_stride;
  const int tid = threadIdx.x;
  const int lane = tid & 63;
  for (int i = tid; i < p; i += 1024) y[i] = (i >= p - nr) ? rhs[i - (p - nr)] : 0.0;
  __syncthreads();
  // forward: L y = e on rows [p-nr, p)
  for (int r0 = p - nr; r0 < p; r0 += 64) {
    const int nbk = min(64, p - r0);
    if (tid < 64) {
      double v = (lane < nbk) ? y[r0 + lane] : 0.0;
      for (int q = 0; q < nbk; ++q) {
        double yq = 0.0;
        if (lane == q) {
          v /= L[(int64_t)(r0 + q) * ld + r0 + q];
        }
        yq = __shfl(v, q, 64);
        if (lane > q && lane < nbk) v -= L[(int64_t)(r0 + lane) * ld + r0 + q] * yq;
      }
      if (lane < nbk) y[r0 + lane] = v;
    }
    __syncthreads();
    for (int r = r0 + nbk + tid; r < p; r += 1024) {
      const double* Lr = L + (int64_t)r * ld + r0;
      double acc = 0.0;
      for (int q = 0; q < nbk; ++q) acc += Lr[q] * y[r0 + q];
      y[r] -= acc;
    }
    __syncthreads();
  }
  // backward: L^T z = y on all rows, bottom-up chunks of 64
  const int nchunk = (p + 63) / 64;
  for (int cidx = nchunk - 1; cidx >= 0; --cidx) {
    const int r0 = cidx * 64;
    const int nbk = min(64, p - r0);
    if (tid < 64) {
      double v = (lane < nbk) ? y[r0 + lane] : 0.0;
      for (int q = nbk - 1; q >= 0; --q) {
        if (lane == q) v /= L[(int64_t)(r0 + q) * ld + r0 + q];
        const double zq = __shfl(v, q, 64);
        if (lane < q) v -= L[(int64_t)(r0 + q) * ld + r0 + lane] * zq;
      }
      if (lane < nbk) y[r0 + lane] = v;
    }
    __syncthreads();
    for (int r = tid; r < r0; r += 1024) {
      double acc = 0.0;
      for (int q = 0; q < nbk; ++q) acc += L[(int64_t)(r0 + q) * ld + r] * y[r0 + q];
      y[r] -= acc;
    }
    __syncthreads();
  }
  for (int i = tid; i < p; i += 1024) z[i] = y[i];
}

}  // namespace

hipError_t launch_cholesky(double* G, int64_t ld, int p, int* info, hipStream_t st) {
  for (int k0 = 0; k0 < p; k0 += kNB) {
    const int nb = min(kNB, p - k0);
    hipLaunchKernelGGL(potrf_diag_kernel, dim3(1), dim3(256), 0, st, G, ld, k0, nb, info);
    const int rest = p - k0 - nb;
    if (rest > 0) {
      hipLaunchKernelGGL(trsm_panel_kernel, dim3((rest + 255) / 256), dim3(256), 0, st, G, ld, k0,
                         nb, p);
      const int T = (rest + 63) / 64;
      hipLaunchKernelGGL(syrk_update_kernel, dim3(T, T), dim3(256), 0, st, G, ld, k0, nb, p);
    }
  }
  return hipGetLastError();
}

hipError_t launch_chol_solve(const double* L, int64_t ld, int p, int nr, const double* rhs64,
                             size_t rhs_stride, double* z, size_t z_stride, int B,
                             hipStream_t st) {
  if (p > kSolveMax) return hipErrorInvalidValue;
  hipLaunchKernelGGL(chol_solve_kernel, dim3(B), dim3(1024), (size_t)p * sizeof(double), st, L, ld,
                     p, nr, rhs64, rhs_stride, z, z_stride);
  return hipGetLastError();
}

}  // namespace slim
