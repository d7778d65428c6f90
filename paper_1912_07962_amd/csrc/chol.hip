// FP64 Cholesky of the Gram system (lambda I + M M^T) and its triangular
// solves, for the explicit-Gram mode (p up to a few thousand).
//
// Blocked right-looking factorisation, panel width 64, row-major lower
// triangle: one workgroup factors a diagonal block in registers and LDS and
// inverts it; the panel below is L21 = A21 L11^{-T} as a GEMM with that
// inverse; the symmetric rank-64 update of the trailing lower triangle runs
// in 64 x 64 tiles.  Look-ahead: the panel kernel also updates the next
// block column, so the next diagonal block is factored in the same launch as
// the rest of the trailing update (one workgroup of that launch), taking the
// update off the chain of dependent diagonal factorisations.  The products
// run on float64 MFMA (v_mfma_f64_16x16x4f64).
//
// The right-hand side [0; ...; 0; res] is zero outside the newest block, so
// the forward solve only touches the trailing rows (one workgroup per
// right-hand side, vector in LDS); the backward solve covers all p rows, one
// launch per diagonal block spread over the rows it updates.  Both use the
// inverses of the diagonal blocks kept by the factorisation.
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
struct PotrfLds {
  double col[2][kNB];
  double piv[kNB];
  double rsq[kNB];   // 1 / sqrt(pivot) = 1 / L[k][k]
  double Ls[kNB][kNB + 1];
  double X[kNB][kNB + 1];   // L^-1 being formed
};
struct TileLds {
  double A[kNB][kNB + 1];
  double B[kNB][kNB + 1];
  double W[kNB][kNB + 1];
};
union CholLds {
  PotrfLds f;
  TileLds t;
};

__device__ __forceinline__ void potrf_diag_body(double* __restrict__ G, int64_t ld, int k0, int nb,
                                                int* __restrict__ info,
                                                double* __restrict__ winv, PotrfLds& S) {
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
      double* cb = S.col[j & 1];
      if (tk == jj) {
#pragma unroll
        for (int m = 0; m < 4; ++m) cb[ti + 16 * m] = a[m][n];
      }
      __syncthreads();
      double d = cb[j];
      const bool bad = !(d > 0.0);  // catches NaN too
      if (bad) d = 1.0;
      if (threadIdx.x == 0) {
        S.piv[j] = d;
        if (bad && info) atomicCAS(info, 0, k0 + j + 1);
      }
      // 1/d from the hardware reciprocal and two Newton steps (each squares
      // the relative error), off the IEEE division's longer dependent chain
      double rd = __builtin_amdgcn_rcp(d);
      rd = fma(rd, fma(-d, rd, 1.0), rd);
      rd = fma(rd, fma(-d, rd, 1.0), rd);
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
  if (threadIdx.x < kNB) S.rsq[threadIdx.x] = (threadIdx.x < nb) ? 1.0 / sqrt(S.piv[threadIdx.x]) : 0.0;
  __syncthreads();
#pragma unroll
  for (int m = 0; m < 4; ++m)
#pragma unroll
    for (int n = 0; n < 4; ++n) {
      const int i = ti + 16 * m, k = tk + 16 * n;
      double v = 0.0;
      if (i < nb && k < i)
        v = a[m][n] * S.rsq[k];
      else if (i < nb && k == i)
        v = sqrt(S.piv[i]);
      S.Ls[i][k] = v;
      if (i < nb && k <= i) G[(int64_t)(k0 + i) * ld + (k0 + k)] = v;
    }
  __syncthreads();
  // L^-1 in 2 x 2 blocks of 32: X11 = L11^-1 and X22 = L22^-1 by
  // substitution (one lane per column, both blocks at once), then
  // X21 = -X22 (L21 X11) by all lanes; X12 = 0.
  constexpr int kH = kNB / 2;
  if (threadIdx.x < kNB) {
    const int c = threadIdx.x & (kH - 1), o = threadIdx.x & kH;
    double w[kH];
#pragma unroll
    for (int i = 0; i < kH; ++i) {
      // four independent partial sums keep the substitution's chain short
      double s4[4] = {(i == c) ? 1.0 : 0.0, 0.0, 0.0, 0.0};
#pragma unroll
      for (int k = 0; k < i; ++k) s4[k & 3] -= S.Ls[o + i][o + k] * w[k];
      w[i] = ((s4[0] + s4[1]) + (s4[2] + s4[3])) * S.rsq[o + i];   // rsq = 0 past nb
    }
#pragma unroll
    for (int i = 0; i < kH; ++i) S.X[o + i][o + c] = w[i];
  }
  __syncthreads();
  // T = L21 X11 into the (zero) upper-right block of X, then
  // X21 = -X22 T.  A lane takes column q of rows r, r + 8, r + 16, r + 24;
  // the sums run over all 32 terms (the triangles' zeros are stored), fully
  // unrolled with four independent accumulators.
  static_assert(kH * kH == 4 * 256, "four entries of each 32 x 32 product per lane");
  const int q = threadIdx.x & (kH - 1), r0 = threadIdx.x >> 5;   // r0 in [0, 8)
  {
    double t[4] = {0.0, 0.0, 0.0, 0.0};
#pragma unroll
    for (int k = 0; k < kH; ++k) {
      const double x = S.X[k][q];
#pragma unroll
      for (int j = 0; j < 4; ++j) t[j] += S.Ls[kH + r0 + 8 * j][k] * x;
    }
#pragma unroll
    for (int j = 0; j < 4; ++j) S.X[r0 + 8 * j][kH + q] = t[j];
  }
  __syncthreads();
  {
    double t[4] = {0.0, 0.0, 0.0, 0.0};
#pragma unroll
    for (int k = 0; k < kH; ++k) {
      const double x = S.X[k][kH + q];
#pragma unroll
      for (int j = 0; j < 4; ++j) t[j] += S.X[kH + r0 + 8 * j][kH + k] * x;
    }
#pragma unroll
    for (int j = 0; j < 4; ++j) S.X[kH + r0 + 8 * j][q] = -t[j];
  }
  __syncthreads();
  for (int e = threadIdx.x; e < kNB * kNB; e += 256) {
    const int i = e / kNB, c = e % kNB;
    winv[e] = (c <= i && c < nb && i < nb) ? S.X[i][c] : 0.0;
  }
}

__global__ __launch_bounds__(256) void potrf_diag_kernel(double* __restrict__ G, int64_t ld, int k0,
                                                         int nb, int* __restrict__ info,
                                                         double* __restrict__ winv) {
  __shared__ CholLds lds;
  potrf_diag_body(G, ld, k0, nb, info, winv, lds.f);
}

typedef double double4_t __attribute__((ext_vector_type(4)));

// acc = A B^T for the 16-row strip w of a 64 x 64 product (K = 64), A and B
// row-major in LDS, on v_mfma_f64_16x16x4f64: A is 16x4 (lane l holds
// A[l%16][l/16]), B is 4x16 (lane l holds B[l/16][l%16]); D is 16x16 and
// accumulator v of lane l holds D[4*v + l/16][l%16] (rows interleaved across
// the accumulators); acc[cb] is the 16 x 16 block of columns 16 cb.
__device__ __forceinline__ void gemm_abt(const double (*A)[kNB + 1], const double (*B)[kNB + 1],
                                         int w, int lane, double4_t acc[4]) {
#pragma unroll
  for (int cb = 0; cb < 4; ++cb) acc[cb] = (double4_t){0.0, 0.0, 0.0, 0.0};
  const int ar = w * 16 + (lane & 15);
  const int kq = lane >> 4;
  for (int k = 0; k < kNB; k += 4) {
    const double av = A[ar][k + kq];
#pragma unroll
    for (int cb = 0; cb < 4; ++cb) {
      const double bv = B[cb * 16 + (lane & 15)][k + kq];
      acc[cb] = __builtin_amdgcn_mfma_f64_16x16x4f64(av, bv, acc[cb], 0, 0, 0);
    }
  }
}

// Panel k and the next block column, one workgroup per 64-row tile i of the
// rows below block k (base = k0 + nb): L_i = A_i W^T with W = L_kk^{-1}
// (stored into the panel), the same for the tile of block k + 1's rows (L_0,
// recomputed by every workgroup), and the update of the tile (i, k + 1):
// G_i,k+1 -= L_i L_0^T (its lower triangle for i = 0).  Every later panel's
// update of block column k + 1 is then complete, so block k + 1 can be
// factored while the rest of panel k's update runs (potrf_syrk_kernel).
__global__ __launch_bounds__(256) void trsm_col_kernel(double* __restrict__ G, int64_t ld, int k0,
                                                       int nb, int p,
                                                       const double* __restrict__ winv) {
  __shared__ CholLds lds;
  TileLds& S = lds.t;
  const int base = k0 + nb;
  const int r0 = base + blockIdx.x * 64;
  {
    // all 48 loads of a lane issued before the first is stored
    double va[16], vb[16], vw[16];
#pragma unroll
    for (int u = 0; u < 16; ++u) {
      const int e = (int)threadIdx.x + 256 * u, r = e / kNB, q = e % kNB;
      const bool okq = q < nb;
      va[u] = (okq && r0 + r < p) ? G[(int64_t)(r0 + r) * ld + k0 + q] : 0.0;
      vb[u] = (okq && base + r < p) ? G[(int64_t)(base + r) * ld + k0 + q] : 0.0;
      vw[u] = winv[e];  // zero outside nb
    }
#pragma unroll
    for (int u = 0; u < 16; ++u) {
      const int e = (int)threadIdx.x + 256 * u, r = e / kNB, q = e % kNB;
      S.A[r][q] = va[u];
      S.B[r][q] = vb[u];
      S.W[r][q] = vw[u];
    }
  }
  __syncthreads();
  const int w = threadIdx.x >> 6;
  const int lane = threadIdx.x & 63;
  double4_t li[4], l0[4];
  gemm_abt(S.A, S.W, w, lane, li);
  gemm_abt(S.B, S.W, w, lane, l0);
  __syncthreads();
#pragma unroll
  for (int cb = 0; cb < 4; ++cb) {
#pragma unroll
    for (int v = 0; v < 4; ++v) {
      const int rr = w * 16 + 4 * v + (lane >> 4);
      const int cc = cb * 16 + (lane & 15);
      S.A[rr][cc] = li[cb][v];
      S.B[rr][cc] = l0[cb][v];
      if (r0 + rr < p && cc < nb) G[(int64_t)(r0 + rr) * ld + k0 + cc] = li[cb][v];
    }
  }
  __syncthreads();
  double4_t up[4];
  gemm_abt(S.A, S.B, w, lane, up);
#pragma unroll
  for (int cb = 0; cb < 4; ++cb) {
#pragma unroll
    for (int v = 0; v < 4; ++v) {
      const int r = r0 + w * 16 + 4 * v + (lane >> 4);
      const int c = base + cb * 16 + (lane & 15);
      if (r < p && c < p && c <= r) G[(int64_t)r * ld + c] -= up[cb][v];
    }
  }
}

// Workgroup (0, 0): factor and invert block k + 1 (rows base .. base + nb1).
// Workgroup (tj, ti), 1 <= tj <= ti: the update of tile (ti, tj) of the
// trailing matrix below block k (tile rows/columns base + 64 ti, base + 64 tj)
// by panel k: A22 -= L21 L21^T.  The two touch disjoint entries; tile column
// 0 (block k + 1's columns) was updated by trsm_col_kernel.
__global__ __launch_bounds__(256) void potrf_syrk_kernel(double* __restrict__ G, int64_t ld,
                                                         int k0, int nb, int p,
                                                         int* __restrict__ info,
                                                         double* __restrict__ winv_next) {
  __shared__ CholLds lds;
  const int ti = blockIdx.y, tj = blockIdx.x;
  const int base = k0 + nb;
  if (ti == 0 && tj == 0) {
    potrf_diag_body(G, ld, base, min(kNB, p - base), info, winv_next, lds.f);
    return;
  }
  if (tj == 0 || tj > ti) return;
  TileLds& S = lds.t;
  const int r0 = base + ti * 64, c0 = base + tj * 64;
  {
    double va[16], vb[16];
#pragma unroll
    for (int u = 0; u < 16; ++u) {
      const int e = (int)threadIdx.x + 256 * u, r = e / kNB, q = e % kNB;
      const bool okq = q < nb;
      va[u] = (okq && r0 + r < p) ? G[(int64_t)(r0 + r) * ld + k0 + q] : 0.0;
      vb[u] = (okq && c0 + r < p) ? G[(int64_t)(c0 + r) * ld + k0 + q] : 0.0;
    }
#pragma unroll
    for (int u = 0; u < 16; ++u) {
      const int e = (int)threadIdx.x + 256 * u, r = e / kNB, q = e % kNB;
      S.A[r][q] = va[u];
      S.B[r][q] = vb[u];
    }
  }
  __syncthreads();
  const int w = threadIdx.x >> 6;
  const int lane = threadIdx.x & 63;
  double4_t acc[4];
  gemm_abt(S.A, S.B, w, lane, acc);
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

// Triangular solves with the inverses W of the 64-row diagonal blocks kept by
// the factorisation, so a block's solve is a 64 x 64 matrix-vector product
// (no dependent chain).  Forward, L y = e: one workgroup per right-hand side
// with the vector in LDS, from the block holding row p - nr (the rows above
// it have a zero right-hand side), so it touches only the trailing rows.
// Backward, L^T z = y on all p rows: one launch per diagonal block, bottom
// up, each spread over the rows it updates (below).
constexpr int kSolveMax = 12288;

__global__ __launch_bounds__(1024) void chol_fwd_kernel(const double* __restrict__ L, int64_t ld,
                                                        int p, int nr,
                                                        const double* __restrict__ winv,
                                                        const double* __restrict__ rhs_all,
                                                        size_t rhs_stride,
                                                        double* __restrict__ y_all,
                                                        size_t y_stride) {
  extern __shared__ double y[];
  __shared__ double Wd[kNB][kNB + 1];
  const double* rhs = rhs_all + (size_t)blockIdx.x * rhs_stride;
  const int tid = threadIdx.x;
  const int first = ((p - nr) / kNB) * kNB;
  for (int i = first + tid; i < p; i += 1024) y[i] = (i >= p - nr) ? rhs[i - (p - nr)] : 0.0;
  for (int r0 = first; r0 < p; r0 += kNB) {
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
    // rows below: 16 lanes per row, 4 consecutive entries each (coalesced),
    // summed across the 16 lanes in a fixed butterfly order
    const int sub = tid & 15;
    for (int rb = r0 + nbk; rb < p; rb += 64) {
      const int r = rb + (tid >> 4);
      double acc = 0.0;
      if (r < p) {
        const double* Lr = L + (int64_t)r * ld + r0;
#pragma unroll
        for (int u = 0; u < 4; ++u) {
          const int q = 4 * sub + u;
          if (q < nbk) acc += Lr[q] * y[r0 + q];
        }
      }
#pragma unroll
      for (int o = 8; o > 0; o >>= 1) acc += __shfl_xor(acc, o, 16);
      if (r < p && sub == 0) y[r] -= acc;
    }
    __syncthreads();
  }
  double* yo = y_all + (size_t)blockIdx.x * y_stride;
  for (int i = tid; i < p; i += 1024) yo[i] = (i >= first) ? y[i] : 0.0;
}

// Backward step for diagonal block c (rows r0 .. r0 + nbk - 1), y final on
// those rows: z_c = W_c^T y_c, written by workgroup 0; every workgroup forms
// z_c itself (same order: same values) and updates its 64 rows r < r0 with
// y[r] -= sum_q L[r0 + q][r] z_c[q] (four partial sums of 16 terms per row,
// added in fixed order).  Grid: (max(1, ceil(r0 / 64)), right-hand sides).
__global__ __launch_bounds__(256) void chol_back_step_kernel(const double* __restrict__ L,
                                                             int64_t ld, int r0, int nbk,
                                                             const double* __restrict__ W,
                                                             double* __restrict__ y_all,
                                                             size_t y_stride,
                                                             double* __restrict__ z_all,
                                                             size_t z_stride) {
  __shared__ double yc[kNB];
  __shared__ double zc[kNB];
  __shared__ double part[4][kNB];
  double* y = y_all + (size_t)blockIdx.y * y_stride;
  const int t = threadIdx.x & (kNB - 1), h = threadIdx.x >> 6;   // 4 quarters of 16 terms
  const int r = blockIdx.x * kNB + t;
  // the lane's W and L entries are requested before y_c arrives
  double wv[16], lv[16];
#pragma unroll
  for (int u = 0; u < 16; ++u) {
    const int q = 16 * h + u;
    wv[u] = (q >= t && q < nbk) ? W[q * kNB + t] : 0.0;
    lv[u] = (r < r0 && q < nbk) ? L[(int64_t)(r0 + q) * ld + r] : 0.0;
  }
  if (threadIdx.x < kNB) yc[t] = (t < nbk) ? y[r0 + t] : 0.0;
  __syncthreads();
  double v = 0.0;
#pragma unroll
  for (int u = 0; u < 16; ++u) v += wv[u] * yc[16 * h + u];
  part[h][t] = v;
  __syncthreads();
  if (threadIdx.x < kNB) {
    const double zt = (part[0][t] + part[1][t]) + (part[2][t] + part[3][t]);
    zc[t] = (t < nbk) ? zt : 0.0;
    if (blockIdx.x == 0 && t < nbk) z_all[(size_t)blockIdx.y * z_stride + r0 + t] = zt;
  }
  __syncthreads();
  double u2 = 0.0;
#pragma unroll
  for (int u = 0; u < 16; ++u) u2 += lv[u] * zc[16 * h + u];
  part[h][t] = u2;
  __syncthreads();
  if (threadIdx.x < kNB && r < r0) y[r] -= (part[0][t] + part[1][t]) + (part[2][t] + part[3][t]);
}


}  // namespace

hipError_t launch_cholesky(double* G, int64_t ld, int p, int* info, double* work,
                           hipStream_t st) {
  if (p <= 0) return hipSuccess;
  int k0 = 0, nb = min(kNB, p);
  hipLaunchKernelGGL(potrf_diag_kernel, dim3(1), dim3(256), 0, st, G, ld, 0, nb, info, work);
  for (;;) {
    const int base = k0 + nb, rest = p - base;
    if (rest <= 0) break;
    const int T = (rest + kNB - 1) / kNB;
    hipLaunchKernelGGL(trsm_col_kernel, dim3(T), dim3(256), 0, st, G, ld, k0, nb, p,
                       (const double*)(work + (size_t)(k0 / kNB) * kNB * kNB));
    hipLaunchKernelGGL(potrf_syrk_kernel, dim3(T, T), dim3(256), 0, st, G, ld, k0, nb, p, info,
                       work + (size_t)(base / kNB) * kNB * kNB);
    k0 = base;
    nb = min(kNB, rest);
  }
  return hipGetLastError();
}

hipError_t launch_chol_solve(const double* L, int64_t ld, int p, int nr, const double* work,
                             const double* rhs64, size_t rhs_stride, double* z, size_t z_stride,
                             double* ywork, int B, hipStream_t st) {
  if (p > kSolveMax) return hipErrorInvalidValue;
  hipLaunchKernelGGL(chol_fwd_kernel, dim3(B), dim3(1024), (size_t)p * sizeof(double), st, L, ld,
                     p, nr, work, rhs64, rhs_stride, ywork, z_stride);
  for (int c = (p + kNB - 1) / kNB - 1; c >= 0; --c) {
    const int r0 = c * kNB, nbk = min(kNB, p - r0);
    hipLaunchKernelGGL(chol_back_step_kernel, dim3(std::max(1, (r0 + kNB - 1) / kNB), B),
                       dim3(256), 0, st, L, ld, r0, nbk, work + (size_t)c * kNB * kNB, ywork,
                       z_stride, z, z_stride);
  }
  return hipGetLastError();
}

}  // namespace slim
