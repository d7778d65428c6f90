// Matrix-free Joseph projectors for gfx950.
//
// Forward (ray-driven): one lane per ray, a 64-wide wavefront covers 64
// adjacent rays of one angle, and the four wavefronts of a workgroup split
// the ray's path into four consecutive segments whose partial sums are
// combined in a fixed order (deterministic).  A ray steps along its major
// axis (rows for |cos| >= |sin|, else columns) and evaluates the canonical
// weight on the three pixels nearest its crossing point; the weight is
// exactly zero on all but at most two of them.  For column-stepping angles
// the transposed image is read when available, so that adjacent lanes read
// adjacent addresses in both cases.
//
// Back (pixel-driven gather): one lane per pixel of a 16x16 tile; for every
// angle of the list the pixel's two rays are read and weighted.  No atomics;
// the optional fused update writes x -= s (and its transpose through LDS)
// and per-workgroup float64 partial norms.
#include "slim_internal.h"
#include "pcg.h"

namespace slim {

namespace {

constexpr int kFwdSeg = 4;

// SQ: accumulate squared weights (row norms of A) instead of weight * pixel.
template <bool SQ>
__global__ __launch_bounds__(256) void forward_kernel(const AngleGeom* __restrict__ geom, int N,
                                                      int R, AngleList ids,
                                                      const float* __restrict__ img,
                                                      const float* __restrict__ imgT,
                                                      const float* __restrict__ sub,
                                                      float* __restrict__ out32,
                                                      double* __restrict__ out64) {
  __shared__ double red[kFwdSeg][64];
  const int lane = threadIdx.x & 63;
  const int seg = threadIdx.x >> 6;
  const int tr = blockIdx.x * 64 + lane;
  const int a = blockIdx.y;
  const int ang = ids.id[a];
  const AngleGeom g = geom[ang];
  const double half = 0.5 * (N - 1);
  const double off = 0.5 * (R - 1);
  double acc = 0.0;
  if (tr < R) {
    const double cm = g.colmajor ? g.c : g.s;  // coefficient of the major coordinate
    const double cn = g.colmajor ? g.s : g.c;  // coefficient of the minor one, |cn| = d
    const double inv = 1.0 / cn;
    const double n0 = ((double)tr - off) * inv;  // crossing minor coordinate at major 0
    const double n1 = -cm * inv;                 // its change per major step
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
    int klo = 0, khi = -1;
    if (lo <= hi) {
      klo = max(0, (int)ceil(lo + half) - 1);
      khi = min(N - 1, (int)floor(hi + half) + 1);
    }
    const int cnt = khi - klo + 1;
    if (cnt > 0) {
      const int per = (cnt + kFwdSeg - 1) / kFwdSeg;
      const int k0 = klo + seg * per;
      const int k1 = min(khi, k0 + per - 1);
      if (!g.colmajor) {
        for (int k = k0; k <= k1; ++k) {
          const double ii = (double)k - half;
          const double inner = fma(ii, g.s, off);
          const double nc = fma(ii, n1, n0) + half;
          const int jc = (int)rint(nc);
          const float* row = img + (size_t)k * N;
          float racc = 0.f;
#pragma unroll
          for (int dj = -1; dj <= 1; ++dj) {
            const int j = jc + dj;
            if (j >= 0 && j < N) {
              const double t = fma((double)j - half, g.c, inner);
              const float w = ray_weight(g, t, tr);
              racc = fmaf(w, SQ ? w : row[j], racc);
            }
          }
          acc += (double)racc;
        }
      } else {
        for (int k = k0; k <= k1; ++k) {
          const double jj = (double)k - half;
          const double nc = fma(jj, n1, n0) + half;
          const int ic = (int)rint(nc);
          float racc = 0.f;
#pragma unroll
          for (int di = -1; di <= 1; ++di) {
            const int i = ic + di;
            if (i >= 0 && i < N) {
              const double t = fma(jj, g.c, fma((double)i - half, g.s, off));
              const float w = ray_weight(g, t, tr);
              const float v = SQ ? w : (imgT ? imgT[(size_t)k * N + i] : img[(size_t)i * N + k]);
              racc = fmaf(w, v, racc);
            }
          }
          acc += (double)racc;
        }
      }
    }
  }
  red[seg][lane] = acc;
  __syncthreads();
  if (seg == 0 && tr < R) {
    double v = red[0][lane];
#pragma unroll
    for (int q = 1; q < kFwdSeg; ++q) v += red[q][lane];
    if (sub) v -= (double)sub[(size_t)ang * R + tr];
    const size_t o = (size_t)a * R + tr;
    if (out32) out32[o] = (float)v;
    if (out64) out64[o] = v;
  }
}

constexpr int kTile = 16;

__device__ __forceinline__ double wave_sum(double v) {
  for (int o = 32; o > 0; o >>= 1) v += __shfl_down(v, o, 64);
  return v;
}

template <typename VT>
__global__ __launch_bounds__(256) void back_kernel(const AngleGeom* __restrict__ geom, int N, int R,
                                                   AngleList ids, const VT* __restrict__ v,
                                                   float* __restrict__ out, float* __restrict__ x,
                                                   float* __restrict__ xT,
                                                   const float* __restrict__ x_true,
                                                   double* __restrict__ partials, int mode) {
  __shared__ float tileT[kTile][kTile + 1];
  __shared__ double wred[4][3];
  const int tx = threadIdx.x & (kTile - 1);
  const int ty = threadIdx.x / kTile;
  const int j = blockIdx.x * kTile + tx;
  const int i = blockIdx.y * kTile + ty;
  const bool in = (i < N) && (j < N);
  const double half = 0.5 * (N - 1);
  const double off = 0.5 * (R - 1);
  const double ii = (double)i - half, jj = (double)j - half;
  float s = 0.f;
  if (in) {
    for (int a = 0; a < ids.n; ++a) {
      const AngleGeom g = geom[ids.id[a]];
      const double t = det_coord(g, ii, jj, off);
      int t0;
      float w0, w1;
      pixel_weights(g, t, t0, w0, w1);
      const VT* va = v + (size_t)a * R;
      const float v0 = (t0 >= 0 && t0 < R) ? (float)va[t0] : 0.f;
      const float v1 = (t0 + 1 >= 0 && t0 + 1 < R) ? (float)va[t0 + 1] : 0.f;
      s = fmaf(w0, v0, s);
      s = fmaf(w1, v1, s);
    }
  }
  if (mode == 0) {
    if (in) out[(size_t)i * N + j] = s;
    if (xT) {  // transposed copy of out through LDS
      tileT[ty][tx] = s;
      __syncthreads();
      const int jt = blockIdx.x * kTile + ty;
      const int it = blockIdx.y * kTile + tx;
      if (jt < N && it < N) xT[(size_t)jt * N + it] = tileT[tx][ty];
    }
    return;
  }
  double ss = 0.0, xx = 0.0, ee = 0.0;
  float xn = 0.f;
  if (in) {
    const size_t p = (size_t)i * N + j;
    xn = x[p] - s;
    x[p] = xn;
    ss = (double)s * (double)s;
    xx = (double)xn * (double)xn;
    if (x_true) {
      const double e = (double)xn - (double)x_true[p];
      ee = e * e;
    }
  }
  if (xT) {
    tileT[ty][tx] = xn;
    __syncthreads();
    // write the transposed tile: lane (ty, tx) writes xT[j'][i'] with
    // j' = tile column ty, i' = tile row tx -> 16 consecutive floats per row
    const int jt = blockIdx.x * kTile + ty;
    const int it = blockIdx.y * kTile + tx;
    if (jt < N && it < N) xT[(size_t)jt * N + it] = tileT[tx][ty];
  }
  ss = wave_sum(ss);
  xx = wave_sum(xx);
  ee = wave_sum(ee);
  const int w = threadIdx.x >> 6;
  if ((threadIdx.x & 63) == 0) {
    wred[w][0] = ss;
    wred[w][1] = xx;
    wred[w][2] = ee;
  }
  __syncthreads();
  if (threadIdx.x < 3) {
    const double r = wred[0][threadIdx.x] + wred[1][threadIdx.x] + wred[2][threadIdx.x] +
                     wred[3][threadIdx.x];
    partials[(size_t)3 * (blockIdx.y * gridDim.x + blockIdx.x) + threadIdx.x] = r;
  }
}

__global__ __launch_bounds__(256) void reduce3_kernel(const double* __restrict__ partials, int n,
                                                      double* __restrict__ out) {
  __shared__ double red[3][256];
  double a0 = 0.0, a1 = 0.0, a2 = 0.0;
  for (int k = threadIdx.x; k < n; k += 256) {
    a0 += partials[3 * (size_t)k + 0];
    a1 += partials[3 * (size_t)k + 1];
    a2 += partials[3 * (size_t)k + 2];
  }
  red[0][threadIdx.x] = a0;
  red[1][threadIdx.x] = a1;
  red[2][threadIdx.x] = a2;
  __syncthreads();
  for (int sz = 128; sz > 0; sz >>= 1) {
    if ((int)threadIdx.x < sz) {
      red[0][threadIdx.x] += red[0][threadIdx.x + sz];
      red[1][threadIdx.x] += red[1][threadIdx.x + sz];
      red[2][threadIdx.x] += red[2][threadIdx.x + sz];
    }
    __syncthreads();
  }
  if (threadIdx.x < 3) out[threadIdx.x] = red[threadIdx.x][0];
}

__global__ __launch_bounds__(256) void transpose_kernel(const float* __restrict__ src,
                                                        float* __restrict__ dst, int N) {
  __shared__ float t[kTile][kTile + 1];
  const int tx = threadIdx.x & (kTile - 1), ty = threadIdx.x / kTile;
  const int i = blockIdx.y * kTile + ty, j = blockIdx.x * kTile + tx;
  if (i < N && j < N) t[ty][tx] = src[(size_t)i * N + j];
  __syncthreads();
  const int jt = blockIdx.x * kTile + ty, it = blockIdx.y * kTile + tx;
  if (jt < N && it < N) dst[(size_t)jt * N + it] = t[tx][ty];
}

}  // namespace

hipError_t launch_forward(const AngleGeom* geom, int N, int R, const AngleList& ids,
                          const float* img, const float* imgT, const float* sub, float* out32,
                          double* out64, hipStream_t st) {
  if (ids.n <= 0) return hipSuccess;
  dim3 grid((R + 63) / 64, ids.n);
  hipLaunchKernelGGL(forward_kernel<false>, grid, dim3(256), 0, st, geom, N, R, ids, img, imgT, sub,
                     out32, out64);
  return hipGetLastError();
}

hipError_t launch_ray_sqnorm(const AngleGeom* geom, int N, int R, const AngleList& ids, double* out,
                             hipStream_t st) {
  if (ids.n <= 0) return hipSuccess;
  dim3 grid((R + 63) / 64, ids.n);
  hipLaunchKernelGGL(forward_kernel<true>, grid, dim3(256), 0, st, geom, N, R, ids, nullptr,
                     nullptr, nullptr, nullptr, out);
  return hipGetLastError();
}

hipError_t launch_transpose(const float* src, float* dst, int N, hipStream_t st) {
  const int t = (N + kTile - 1) / kTile;
  hipLaunchKernelGGL(transpose_kernel, dim3(t, t), dim3(256), 0, st, src, dst, N);
  return hipGetLastError();
}

int back_num_workgroups(int N) {
  const int t = (N + kTile - 1) / kTile;
  return t * t;
}

hipError_t launch_back(const AngleGeom* geom, int N, int R, const AngleList& ids,
                       const float* v32, const double* v64, float* out, float* x, float* xT,
                       const float* x_true, double* partials, int mode, hipStream_t st) {
  const int t = (N + kTile - 1) / kTile;
  dim3 grid(t, t);
  if (v64) {
    hipLaunchKernelGGL(back_kernel<double>, grid, dim3(256), 0, st, geom, N, R, ids, v64, out, x,
                       xT, x_true, partials, mode);
  } else {
    hipLaunchKernelGGL(back_kernel<float>, grid, dim3(256), 0, st, geom, N, R, ids, v32, out, x,
                       xT, x_true, partials, mode);
  }
  return hipGetLastError();
}

hipError_t launch_reduce3(const double* partials, int n, double* out, hipStream_t st) {
  hipLaunchKernelGGL(reduce3_kernel, dim3(1), dim3(256), 0, st, partials, n, out);
  return hipGetLastError();
}

}  // namespace slim
