// FP64 Cholesky of the Gram system (lambda I + M M^T) and its triangular
// solves, for the explicit-Gram mode (p up to a few thousand).
//
// Blocked right-looking factorisation, panel width 64, row-major lower
// triangle: per panel one workgroup factors the diagonal block in LDS and
// inverts it, the panel below is L21 = A21 L11^{-T} as a GEMM with that
// inverse, and a tiled kernel applies the symmetric rank-64 update to the
// trailing lower triangle; both products run on float64 MFMA
// (v_mfma_f64_16x16x4f64).
//
// The right-hand side [0; ...; 0; res] is zero outside the newest block, so
// the forward solve only touches the trailing rows; the backward solve covers
// all p rows.  Both run in one workgroup per right-hand side with the vector
// in LDS, using the inverses of the diagonal blocks kept by the factorisation.
#include "slim_internal.h"

namespace slim {

namespace {

constexpr int kNB = 64;

// Factor the diagonal block and invert it.  Factorisation: thread (ti, tk)
// of a 16 x 16 grid holds entries (ti + 16m, tk + 16n), m, n < 4, of the
// block in registers for the whole right-looking elimination; at pivot j
// the owners of column j publish it through a double-buffered LDS vector (one
// barrier per pivot) and every thread updates its entries with the unscaled
// column divided by the pivot; the square roots are applied at the end.
// Inverse W = L11^{-1}: one wavefront, lane c substitutes column c with the
// column held in registers and L read by LDS broadcast.  W goes to winv for
// the panel GEMM and the triangular solves.
__global__ __launch_bounds__(256) void potrf_diag_kernel(double* __restrict__ G, int64_t ld, int k0,
                                                         int nb, int* __restrict__ info,
                                                         double* __restrict__ winv) {
  __shared__ double col[2][kNB];
  __shared__ double piv[kNB];
  __shared__ double Ls[kNB][kNB + 1];
  const int ti = threadIdx.x >> 4, tk = threadIdx.x & 15;
  double a[4][4];
#pragma unroll
  for (int m = 0; m < 4; ++m)
#pragma unroll
    for (int n = 0; n < 4; ++n) {
      const int i = ti + 16 * m, k = tk + 16 * n;
      a[m][n] = (i < nb && k <= i) ? G[(int64_t)(k0 + i) * ld + (k0 + k)] : 0.0;
    }
#pragma unroll
  for (int n = 0; n < 4; ++n) {
    for (int jj = 0; jj < 16; ++jj) {
      const int j = 16 * n + jj;
      if (j >= nb) break;
      double* cb = col[j & 1];
      if (tk == jj) {
#pragma unroll
        for (int m = 0; m < 4; ++m) cb[ti + 16 * m] = a[m][n];
      }
      __syncthreads();
      double d = cb[j];
      const bool bad = !(d > 0.0);  // catches NaN too
      if (bad) d = 1.0;
      if (threadIdx.x == 0) {
        piv[j] = d;
        if (bad && info) atomicCAS(info, 0, k0 + j + 1);
      }
      const double rd = 1.0 / d;
      double ci[4], ck[4];
#pragma unroll
      for (int m = 0; m < 4; ++m) ci[m] = cb[ti + 16 * m] * rd;
#pragma unroll
      for (int q = 0; q < 4; ++q) ck[q] = cb[tk + 16 * q];
#pragma unroll
      for (int m = 0; m < 4; ++m)
#pragma unroll
        for (int q = 0; q < 4; ++q) {
          const int i = ti + 16 * m, k = tk + 16 * q;
          if (k > j && k <= i) a[m][q] -= ci[m] * ck[q];
        }
    }
  }
  __syncthreads();
#pragma unroll
  for (int m = 0; m < 4; ++m)
#pragma unroll
    for (int n = 0; n < 4; ++n) {
      const int i = ti + 16 * m, k = tk + 16 * n;
      double v = 0.0;
      if (i < nb && k < i)
        v = a[m][n] / sqrt(piv[k]);
      else if (i < nb && k == i)
        v = sqrt(piv[i]);
      Ls[i][k] = v;
      if (i < nb && k <= i) G[(int64_t)(k0 + i) * ld + (k0 + k)] = v;
    }
  __syncthreads();
  if (threadIdx.x < kNB) {
    const int c = threadIdx.x;
    double w[kNB];
#pragma unroll
    for (int i = 0; i < kNB; ++i) {
      double s = (i == c) ? 1.0 : 0.0;
#pragma unroll
      for (int k = 0; k < i; ++k) s -= Ls[i][k] * w[k];
      w[i] = (i < nb) ? s / Ls[i][i] : 0.0;
    }
#pragma unroll
    for (int i = 0; i < kNB; ++i) winv[i * kNB + c] = (c < nb) ? w[i] : 0.0;
  }
}

typedef double double4_t __attribute__((ext_vector_type(4)));

// rows [k0+nb, p), 64 per workgroup: L21 = A21 W^T with W = L11^{-1}, on
// float64 MFMA (4 wavefronts, each a 16-row strip of four 16x16 blocks).
__global__ __launch_bounds__(256) void trsm_gemm_kernel(double* __restrict__ G, int64_t ld, int k0,
                                                        int nb, int p,
                                                        const double* __restrict__ winv) {
  __shared__ double Ai[64][kNB + 1];
  __shared__ double Wj[kNB][kNB + 1];
  const int r0 = k0 + nb + blockIdx.x * 64;
  for (int e = threadIdx.x; e < 64 * kNB; e += 256) {
    const int r = e / kNB, q = e % kNB;
    Ai[r][q] = (q < nb && r0 + r < p) ? G[(int64_t)(r0 + r) * ld + k0 + q] : 0.0;
    Wj[r][q] = winv[e];  // zero outside nb
  }
  __syncthreads();
  const int w = threadIdx.x >> 6;
  const int lane = threadIdx.x & 63;
  double4_t acc[4];
#pragma unroll
  for (int cb = 0; cb < 4; ++cb) acc[cb] = (double4_t){0.0, 0.0, 0.0, 0.0};
  const int ar = w * 16 + (lane & 15);
  const int kq = lane >> 4;
  for (int k = 0; k < kNB; k += 4) {
    const double av = Ai[ar][k + kq];
#pragma unroll
    for (int cb = 0; cb < 4; ++cb) {
      const double bv = Wj[cb * 16 + (lane & 15)][k + kq];
      acc[cb] = __builtin_amdgcn_mfma_f64_16x16x4f64(av, bv, acc[cb], 0, 0, 0);
    }
  }
#pragma unroll
  for (int cb = 0; cb < 4; ++cb) {
#pragma unroll
    for (int v = 0; v < 4; ++v) {
      const int r = r0 + w * 16 + 4 * v + (lane >> 4);
      const int cc = cb * 16 + (lane & 15);
      if (r < p && cc < nb) G[(int64_t)r * ld + k0 + cc] = acc[cb][v];
    }
  }
}

// Trailing update A22 -= L21 L21^T on 64x64 lower tiles, K = nb <= 64.
// 4 wavefronts; wavefront w computes the 16-row strip w of the tile as four
// 16x16 MFMA blocks.

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

// Triangular solves, one workgroup per right-hand side, vector in LDS.  The
// factorisation kept the inverse W of every 64-row diagonal block, so a
// block's solve is a 64 x 64 matrix-vector product (no dependent chain);
// the updates of the remaining rows are row- (forward) or column-coalesced
// (backward).  The forward solve starts at the block holding row p - nr (the
// rows above it have a zero right-hand side).
constexpr int kSolveMax = 12288;

// sum_{q < n} a[q * stride] * v[q] with eight independent partial sums, so
// eight loads are in flight per lane (the order is fixed: deterministic)
__device__ __forceinline__ double dot_rows(const double* __restrict__ a, int64_t stride,
                                           const double* v, int n) {
  double acc[8] = {0.0, 0.0, 0.0, 0.0, 0.0, 0.0, 0.0, 0.0};
  int q = 0;
  for (; q + 8 <= n; q += 8) {
#pragma unroll
    for (int u = 0; u < 8; ++u) acc[u] += a[(q + u) * stride] * v[q + u];
  }
  for (int u = 0; q < n; ++q, ++u) acc[u] += a[q * stride] * v[q];
  return ((acc[0] + acc[1]) + (acc[2] + acc[3])) + ((acc[4] + acc[5]) + (acc[6] + acc[7]));
}

__global__ __launch_bounds__(1024) void chol_solve_kernel(const double* __restrict__ L, int64_t ld,
                                                          int p, int nr,
                                                          const double* __restrict__ winv,
                                                          const double* __restrict__ rhs_all,
                                                          size_t rhs_stride,
                                                          double* __restrict__ z_all,
                                                          size_t z_stride) {
  extern __shared__ double y[];
  __shared__ double Wd[kNB][kNB + 1];
  const double* rhs = rhs_all + (size_t)blockIdx.x * rhs_stride;
  double* z = z_all + (size_t)blockIdx.x * z_stride;
  const int tid = threadIdx.x;
  for (int i = tid; i < p; i += 1024) y[i] = (i >= p - nr) ? rhs[i - (p - nr)] : 0.0;
  // forward: L y = e from the block holding row p - nr
  for (int r0 = ((p - nr) / kNB) * kNB; r0 < p; r0 += kNB) {
    const int nbk = min(kNB, p - r0);
    const double* W = winv + (size_t)(r0 / kNB) * kNB * kNB;
    for (int e = tid; e < kNB * kNB; e += 1024) Wd[e / kNB][e % kNB] = W[e];
    __syncthreads();
    double v = 0.0;
    if (tid < nbk)
      for (int q = 0; q <= tid; ++q) v += Wd[tid][q] * y[r0 + q];
    __syncthreads();
    if (tid < nbk) y[r0 + tid] = v;
    __syncthreads();
    for (int r = r0 + nbk + tid; r < p; r += 1024) {
      const double* Lr = L + (int64_t)r * ld + r0;
      y[r] -= dot_rows(Lr, 1, y + r0, nbk);
    }
    __syncthreads();
  }
  // backward: L^T z = y on all rows, bottom-up blocks
  const int nchunk = (p + kNB - 1) / kNB;
  for (int cidx = nchunk - 1; cidx >= 0; --cidx) {
    const int r0 = cidx * kNB;
    const int nbk = min(kNB, p - r0);
    const double* W = winv + (size_t)cidx * kNB * kNB;
    for (int e = tid; e < kNB * kNB; e += 1024) Wd[e / kNB][e % kNB] = W[e];
    __syncthreads();
    double v = 0.0;
    if (tid < nbk)
      for (int q = tid; q < nbk; ++q) v += Wd[q][tid] * y[r0 + q];
    __syncthreads();
    if (tid < nbk) y[r0 + tid] = v;
    __syncthreads();
    for (int r = tid; r < r0; r += 1024) y[r] -= dot_rows(L + (int64_t)r0 * ld + r, ld, y + r0, nbk);
    __syncthreads();
  }
  for (int i = tid; i < p; i += 1024) z[i] = y[i];
}

}  // namespace

hipError_t launch_cholesky(double* G, int64_t ld, int p, int* info, double* work,
                           hipStream_t st) {
  for (int k0 = 0; k0 < p; k0 += kNB) {
    const int nb = min(kNB, p - k0);
    double* w = work + (size_t)(k0 / kNB) * kNB * kNB;
    hipLaunchKernelGGL(potrf_diag_kernel, dim3(1), dim3(256), 0, st, G, ld, k0, nb, info, w);
    const int rest = p - k0 - nb;
    if (rest > 0) {
      hipLaunchKernelGGL(trsm_gemm_kernel, dim3((rest + 63) / 64), dim3(256), 0, st, G, ld, k0, nb,
                         p, (const double*)w);
      const int T = (rest + 63) / 64;
      hipLaunchKernelGGL(syrk_update_kernel, dim3(T, T), dim3(256), 0, st, G, ld, k0, nb, p);
    }
  }
  return hipGetLastError();
}

hipError_t launch_chol_solve(const double* L, int64_t ld, int p, int nr, const double* work,
                             const double* rhs64, size_t rhs_stride, double* z, size_t z_stride,
                             int B, hipStream_t st) {
  if (p > kSolveMax) return hipErrorInvalidValue;
  hipLaunchKernelGGL(chol_solve_kernel, dim3(B), dim3(1024), (size_t)p * sizeof(double), st, L, ld,
                     p, nr, work, rhs64, rhs_stride, z, z_stride);
  return hipGetLastError();
}

}  // namespace slim
