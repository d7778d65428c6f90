// Jacobi-preconditioned conjugate gradients on (lambda I + M M^T) z = e,
// e = [0; ...; 0; res], for one slice.  Per iteration:
//   u = M^T pd (back-projector, float32 image and its transpose)
//   q = M u (forward projector, float64 sums) ; q += lambda pd ; <pd, q>
//   alpha = rz / <pd, q>            (device scalar)
//   z += alpha pd ; r -= alpha q ; y = D^{-1} r ; <r, y>, <r, r>
//   beta = <r,y>_new / rz ; pd = y + beta pd
// All dot products are two-stage fixed-order reductions (deterministic).
// The host reads ||r|| every kCheck iterations to stop.
#include "pcg.h"

#include <algorithm>
#include <cmath>

namespace slim {

namespace {

constexpr int kThreads = 256;
constexpr int kCheck = 4;

enum { S_RZ = 0, S_ALPHA, S_BETA, S_RR, S_PQ, S_BB, S_COUNT };

__device__ __forceinline__ double block_sum(double v, double* sh) {
  for (int o = 32; o > 0; o >>= 1) v += __shfl_down(v, o, 64);
  const int w = threadIdx.x >> 6;
  if ((threadIdx.x & 63) == 0) sh[w] = v;
  __syncthreads();
  double r = 0.0;
  if (threadIdx.x == 0)
    for (int q = 0; q < kThreads / 64; ++q) r += sh[q];
  __syncthreads();
  return r;
}

// index of the Jacobi entry for p-space row i: angle ids[i / R], ray i % R
__device__ __forceinline__ double dinv_at(const double* dinv, const AngleList& win, int R, int i) {
  return dinv[(size_t)win.id[i / R] * R + (i % R)];
}

// r = e, z = 0, y = D^{-1} r, pd = y; partial <r,y>, <r,r>
__global__ __launch_bounds__(kThreads) void init_kernel(AngleList win, int R, int p, int nres,
                                                        const double* __restrict__ res,
                                                        const double* __restrict__ dinv,
                                                        double* __restrict__ r,
                                                        double* __restrict__ z,
                                                        double* __restrict__ y,
                                                        double* __restrict__ pd,
                                                        double* __restrict__ parts, int nparts) {
  __shared__ double sh[kThreads / 64];
  const int i = blockIdx.x * kThreads + threadIdx.x;
  double ry = 0.0, rr = 0.0;
  if (i < p) {
    const double e = (i >= p - nres) ? res[i - (p - nres)] : 0.0;
    const double yy = dinv_at(dinv, win, R, i) * e;
    r[i] = e;
    z[i] = 0.0;
    y[i] = yy;
    pd[i] = yy;
    ry = e * yy;
    rr = e * e;
  }
  ry = block_sum(ry, sh);
  rr = block_sum(rr, sh);
  if (threadIdx.x == 0) {
    parts[blockIdx.x] = ry;
    parts[nparts + blockIdx.x] = rr;
  }
}

// which: 0 -> init (rz, rr, bb=rr), 1 -> alpha = rz / pq, 2 -> beta, rz, rr
__global__ __launch_bounds__(kThreads) void scalar_kernel(const double* __restrict__ parts,
                                                          int nparts, int which,
                                                          double* __restrict__ sc) {
  __shared__ double sh[kThreads / 64];
  double a = 0.0, b = 0.0;
  for (int k = threadIdx.x; k < nparts; k += kThreads) {
    a += parts[k];
    if (which != 1) b += parts[nparts + k];
  }
  a = block_sum(a, sh);
  b = block_sum(b, sh);
  if (threadIdx.x == 0) {
    if (which == 0) {
      sc[S_RZ] = a;
      sc[S_RR] = b;
      sc[S_BB] = b;
    } else if (which == 1) {
      sc[S_PQ] = a;
      sc[S_ALPHA] = (a != 0.0) ? sc[S_RZ] / a : 0.0;
    } else {
      const double rz = sc[S_RZ];
      sc[S_BETA] = (rz != 0.0) ? a / rz : 0.0;
      sc[S_RZ] = a;
      sc[S_RR] = b;
    }
  }
}

// z += alpha pd; r -= alpha q; y = D^{-1} r; partial <r,y>, <r,r>
__global__ __launch_bounds__(kThreads) void update_kernel(AngleList win, int R, int p,
                                                          const double* __restrict__ sc,
                                                          const double* __restrict__ dinv,
                                                          const double* __restrict__ pd,
                                                          const double* __restrict__ q,
                                                          double* __restrict__ z,
                                                          double* __restrict__ r,
                                                          double* __restrict__ y,
                                                          double* __restrict__ parts, int nparts) {
  __shared__ double sh[kThreads / 64];
  const int i = blockIdx.x * kThreads + threadIdx.x;
  const double alpha = sc[S_ALPHA];
  double ry = 0.0, rr = 0.0;
  if (i < p) {
    z[i] = fma(alpha, pd[i], z[i]);
    const double rn = fma(-alpha, q[i], r[i]);
    r[i] = rn;
    const double yy = dinv_at(dinv, win, R, i) * rn;
    y[i] = yy;
    ry = rn * yy;
    rr = rn * rn;
  }
  ry = block_sum(ry, sh);
  rr = block_sum(rr, sh);
  if (threadIdx.x == 0) {
    parts[blockIdx.x] = ry;
    parts[nparts + blockIdx.x] = rr;
  }
}

// pd = y + beta pd
__global__ __launch_bounds__(kThreads) void direction_kernel(int p, const double* __restrict__ sc,
                                                             const double* __restrict__ y,
                                                             double* __restrict__ pd) {
  const int i = blockIdx.x * kThreads + threadIdx.x;
  if (i < p) pd[i] = fma(sc[S_BETA], pd[i], y[i]);
}

__global__ __launch_bounds__(kThreads) void dinv_kernel(double* __restrict__ d, int n, double lam) {
  const int i = blockIdx.x * kThreads + threadIdx.x;
  if (i < n) d[i] = 1.0 / (d[i] + lam);
}

}  // namespace

hipError_t pcg_alloc(PcgWork& w, int N, int n_angles, int R, int64_t pmax) {
  hipError_t e;
  w.pmax = (int)pmax;
  w.nparts = (int)((pmax + kThreads - 1) / kThreads);
  const size_t np = (size_t)pmax * sizeof(double);
  if ((e = hipMalloc((void**)&w.r, np)) != hipSuccess) return e;
  if ((e = hipMalloc((void**)&w.pd, np)) != hipSuccess) return e;
  if ((e = hipMalloc((void**)&w.q, np)) != hipSuccess) return e;
  if ((e = hipMalloc((void**)&w.y, np)) != hipSuccess) return e;
  if ((e = hipMalloc((void**)&w.dinv, (size_t)n_angles * R * sizeof(double))) != hipSuccess) return e;
  if ((e = hipMalloc((void**)&w.parts, (size_t)2 * w.nparts * sizeof(double))) != hipSuccess) return e;
  if ((e = hipMalloc((void**)&w.sc, S_COUNT * sizeof(double))) != hipSuccess) return e;
  if ((e = hipMalloc((void**)&w.u, (size_t)N * N * sizeof(float))) != hipSuccess) return e;
  if ((e = hipMalloc((void**)&w.uT, (size_t)N * N * sizeof(float))) != hipSuccess) return e;
  if ((e = hipHostMalloc((void**)&w.h_sc, S_COUNT * sizeof(double), hipHostMallocDefault)) != hipSuccess)
    return e;
  return hipSuccess;
}

void pcg_free(PcgWork& w) {
  (void)hipFree(w.r);
  (void)hipFree(w.pd);
  (void)hipFree(w.q);
  (void)hipFree(w.y);
  (void)hipFree(w.dinv);
  (void)hipFree(w.parts);
  (void)hipFree(w.sc);
  (void)hipFree(w.u);
  (void)hipFree(w.uT);
  if (w.h_sc) (void)hipHostFree(w.h_sc);
  w = PcgWork{};
}

hipError_t pcg_setup(PcgWork& w, const AngleGeom* geom, const AngleGeom* h_geom, int N,
                     int n_angles, int R, double lam, float* partial, hipStream_t st) {
  for (int a0 = 0; a0 < n_angles; a0 += kMaxList) {
    AngleList l;
    l.n = std::min(kMaxList, n_angles - a0);
    for (int i = 0; i < kMaxList; ++i) l.id[i] = (i < l.n) ? a0 + i : 0;
    hipError_t e = launch_ray_sqnorm(geom, h_geom, N, R, l, w.dinv + (size_t)a0 * R, partial, st);
    if (e != hipSuccess) return e;
  }
  const int n = n_angles * R;
  hipLaunchKernelGGL(dinv_kernel, dim3((n + kThreads - 1) / kThreads), dim3(kThreads), 0, st, w.dinv,
                     n, lam);
  return hipGetLastError();
}

hipError_t pcg_solve(PcgWork& w, const AngleGeom* geom, const AngleGeom* h_geom, float* partial,
                     int N, int R, const AngleList& win,
                     double lam, const double* res, int nres, double* z, double tol, int max_iter,
                     int* iters, double* relres, Profiler* prof, hipStream_t st) {
  const int p = win.n * R;
  const int nb = (p + kThreads - 1) / kThreads;
  hipError_t e;
  hipLaunchKernelGGL(init_kernel, dim3(nb), dim3(kThreads), 0, st, win, R, p, nres, res, w.dinv,
                     w.r, z, w.y, w.pd, w.parts, nb);
  hipLaunchKernelGGL(scalar_kernel, dim3(1), dim3(kThreads), 0, st, w.parts, nb, 0, w.sc);
  if ((e = hipMemcpyAsync(w.h_sc, w.sc, S_COUNT * sizeof(double), hipMemcpyDeviceToHost, st)) != hipSuccess)
    return e;
  if ((e = hipStreamSynchronize(st)) != hipSuccess) return e;
  const double bb = w.h_sc[S_BB];
  *iters = 0;
  *relres = 0.0;
  if (!(bb > 0.0)) return hipSuccess;
  const double target = tol * tol * bb;
  int it = 0;
  double rr = bb;
  while (it < max_iter) {
    const int todo = std::min(kCheck, max_iter - it);
    for (int q = 0; q < todo; ++q) {
      if (prof->on && (e = prof->begin(K_BACK, st)) != hipSuccess) return e;
      if ((e = launch_back(geom, N, R, win, nullptr, w.pd, w.u, nullptr, w.uT, nullptr, nullptr, 0,
                           st)) != hipSuccess)
        return e;
      if (prof->on && (e = prof->end(st)) != hipSuccess) return e;
      if (prof->on && (e = prof->begin(K_FORWARD, st)) != hipSuccess) return e;
      // q = M u + lambda pd and partial <pd, q>, fused into the forward's reduction
      if ((e = launch_forward(geom, h_geom, N, R, win, w.u, w.uT, nullptr, nullptr, w.q, partial,
                              w.pd, lam, w.parts, st)) != hipSuccess)
        return e;
      if (prof->on && (e = prof->end(st)) != hipSuccess) return e;
      if (prof->on && (e = prof->begin(K_VEC, st)) != hipSuccess) return e;
      hipLaunchKernelGGL(scalar_kernel, dim3(1), dim3(kThreads), 0, st, w.parts, nb, 1, w.sc);
      hipLaunchKernelGGL(update_kernel, dim3(nb), dim3(kThreads), 0, st, win, R, p, w.sc, w.dinv,
                         w.pd, w.q, z, w.r, w.y, w.parts, nb);
      hipLaunchKernelGGL(scalar_kernel, dim3(1), dim3(kThreads), 0, st, w.parts, nb, 2, w.sc);
      hipLaunchKernelGGL(direction_kernel, dim3(nb), dim3(kThreads), 0, st, p, w.sc, w.y, w.pd);
      if ((e = hipGetLastError()) != hipSuccess) return e;
      if (prof->on && (e = prof->end(st)) != hipSuccess) return e;
    }
    it += todo;
    if ((e = hipMemcpyAsync(w.h_sc, w.sc, S_COUNT * sizeof(double), hipMemcpyDeviceToHost, st)) !=
        hipSuccess)
      return e;
    if ((e = hipStreamSynchronize(st)) != hipSuccess) return e;
    if (prof->on && (e = prof->harvest()) != hipSuccess) return e;
    rr = w.h_sc[S_RR];
    if (!(rr > target)) break;  // also stops on NaN
  }
  *iters = it;
  *relres = std::sqrt(rr / bb);
  return hipSuccess;
}

hipError_t Profiler::begin(int k, hipStream_t st) {
  if ((size_t)(2 * used + 2) > pool.size()) {
    for (int q = 0; q < 64; ++q) {
      hipEvent_t ev;
      hipError_t e = hipEventCreate(&ev);
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
