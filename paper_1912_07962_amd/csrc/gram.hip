// Exact Gram blocks A_a A_b^T of the Joseph projector (float64 accumulate).
//
// One lane per entry ((a, t), (b, u)).  The lane walks ray (a, t) along its
// major axis, restricted to the steps whose pixels can reach ray (b, u):
// along ray (a, t) the detector coordinate of angle b is affine in the step,
// t_b = beta + alpha * step, and a pixel within 1.5 of the crossing point can
// only touch ray u while |t_b - u| < 2.5.  Each visited pixel multiplies the
// canonical weights of both rays, so the block is the Gram of the same
// float32 weights the projectors apply.  Same-angle blocks come out
// tridiagonal; non-crossing ray pairs exit at once.
#include "slim_internal.h"

namespace slim {

namespace {

constexpr int kGT = 16;

__global__ __launch_bounds__(256) void gram_kernel(const AngleGeom* __restrict__ geom, int N, int R,
                                                   AngleList ida, AngleList idb,
                                                   double* __restrict__ out, int64_t ld) {
  const int col = blockIdx.x * kGT + (threadIdx.x % kGT);
  const int row = blockIdx.y * kGT + (threadIdx.x / kGT);
  if (row >= ida.n * R || col >= idb.n * R) return;
  const int a = row / R, t = row % R;
  const int b = col / R, u = col % R;
  const AngleGeom ga = geom[ida.id[a]];
  const AngleGeom gb = geom[idb.id[b]];
  const double half = 0.5 * (N - 1);
  const double off = 0.5 * (R - 1);

  const double cm = ga.colmajor ? ga.c : ga.s;
  const double cn = ga.colmajor ? ga.s : ga.c;
  const double inv = 1.0 / cn;
  const double n0 = ((double)t - off) * inv;
  const double n1 = -cm * inv;
  // own in-grid range of ray (a, t)
  const double lim = half + 1.5;
  double lo = -half, hi = half;
  if (n1 != 0.0) {
    const double ma = (-lim - n0) / n1, mb = (lim - n0) / n1;
    lo = fmax(lo, fmin(ma, mb));
    hi = fmin(hi, fmax(ma, mb));
  } else if (fabs(n0) > lim) {
    lo = 1.0;
    hi = 0.0;
  }
  // reach of ray (b, u)
  double alpha, beta;
  if (!ga.colmajor) {  // major = ii, minor = jj = n0 + n1 ii
    alpha = fma(n1, gb.c, gb.s);
    beta = fma(n0, gb.c, off);
  } else {             // major = jj, minor = ii = n0 + n1 jj
    alpha = fma(n1, gb.s, gb.c);
    beta = fma(n0, gb.s, off);
  }
  const double du = (double)u - beta;
  if (fabs(alpha) > 1e-12) {
    const double ma = (du - 2.5) / alpha, mb = (du + 2.5) / alpha;
    lo = fmax(lo, fmin(ma, mb));
    hi = fmin(hi, fmax(ma, mb));
  } else if (fabs(du) >= 2.5) {
    lo = 1.0;
    hi = 0.0;
  }
  double acc = 0.0;
  if (lo <= hi) {
    const int klo = max(0, (int)ceil(lo + half) - 1);
    const int khi = min(N - 1, (int)floor(hi + half) + 1);
    for (int k = klo; k <= khi; ++k) {
      const double mm = (double)k - half;
      const int cc = (int)rint(fma(mm, n1, n0) + half);
#pragma unroll
      for (int d = -1; d <= 1; ++d) {
        const int q = cc + d;
        if (q < 0 || q >= N) continue;
        const double ii = ga.colmajor ? (double)q - half : mm;
        const double jj = ga.colmajor ? mm : (double)q - half;
        const float wa = ray_weight(ga, det_coord(ga, ii, jj, off), t);
        if (wa == 0.f) continue;
        const float wb = ray_weight(gb, det_coord(gb, ii, jj, off), u);
        acc = fma((double)wa, (double)wb, acc);
      }
    }
  }
  out[(int64_t)row * ld + col] = acc;
}

__global__ void tile_copy_kernel(const double* __restrict__ src, int64_t lds, double* __restrict__ G,
                                 int64_t ldg, int r0, int c0, int rows, int cols, double diag,
                                 int add_diag) {
  const int c = blockIdx.x * blockDim.x + threadIdx.x;
  const int r = blockIdx.y;
  if (c >= cols || r >= rows) return;
  double v = src[(int64_t)r * lds + c];
  if (add_diag && r == c) v += diag;
  G[(int64_t)(r0 + r) * ldg + (c0 + c)] = v;
}

// All tiles of the lower triangle of G in one launch: blockIdx.z enumerates
// the window pairs P >= Q (z = P (P + 1) / 2 + Q); window position P holds
// ring slot (first + P) mod S; tile (sp, sq) of the ring is
// tiles[(sp S + sq) ell^2], row-major ell x ell.  lambda goes on G's diagonal.
__global__ void tile_assemble_kernel(const double* __restrict__ tiles, int S, int first, int ell,
                                     double* __restrict__ G, int64_t ldg, double lam) {
  const int c = blockIdx.x * blockDim.x + threadIdx.x;
  const int r = blockIdx.y;
  if (c >= ell) return;
  const int z = blockIdx.z;
  int P = (int)((sqrt(8.0 * z + 1.0) - 1.0) * 0.5);
  while ((P + 1) * (P + 2) / 2 <= z) ++P;   // guard the float estimate
  while (P * (P + 1) / 2 > z) --P;
  const int Q = z - P * (P + 1) / 2;
  const int sp = (first + P) % S, sq = (first + Q) % S;
  const double* T = tiles + ((int64_t)sp * S + sq) * ell * ell;
  double v = T[(int64_t)r * ell + c];
  if (P == Q && r == c) v += lam;
  G[(int64_t)(P * ell + r) * ldg + (Q * ell + c)] = v;
}

}  // namespace

hipError_t launch_tile_assemble(const double* tiles, int S, int first, int W, int ell, double* G,
                                int64_t ldg, double lam, hipStream_t st) {
  const int64_t pairs = (int64_t)W * (W + 1) / 2;
  if (pairs == 0 || ell == 0) return hipSuccess;
  if (pairs > 65535 || ell > 65535) return hipErrorInvalidValue;
  dim3 grid((ell + 255) / 256, ell, (unsigned)pairs);
  hipLaunchKernelGGL(tile_assemble_kernel, grid, dim3(256), 0, st, tiles, S, first, ell, G, ldg,
                     lam);
  return hipGetLastError();
}

hipError_t launch_gram(const AngleGeom* geom, int N, int R, const AngleList& ida,
                       const AngleList& idb, double* out, int64_t ld, hipStream_t st) {
  const int rows = ida.n * R, cols = idb.n * R;
  if (rows == 0 || cols == 0) return hipSuccess;
  dim3 grid((cols + kGT - 1) / kGT, (rows + kGT - 1) / kGT);
  hipLaunchKernelGGL(gram_kernel, grid, dim3(kGT * kGT), 0, st, geom, N, R, ida, idb, out, ld);
  return hipGetLastError();
}

hipError_t launch_tile_copy(const double* src, int64_t lds, double* G, int64_t ldg, int r0, int c0,
                            int rows, int cols, double diag, int add_diag, hipStream_t st) {
  if (rows == 0 || cols == 0) return hipSuccess;
  dim3 grid((cols + 255) / 256, rows);
  hipLaunchKernelGGL(tile_copy_kernel, grid, dim3(256), 0, st, src, lds, G, ldg, r0, c0, rows, cols,
                     diag, add_diag);
  return hipGetLastError();
}

}  // namespace slim
