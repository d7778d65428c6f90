// Conjugate gradients on the Gram system (lambda I + M M^T) z = e,
// e = [0; ...; 0; res], for one slice, with matrix-free M and M^T.
// Per iteration:
//   u = M^T pd                 back-projector (float32 image and transpose)
//   q = M u + lambda pd        forward projector, float64 sums, with the
//                              partial sums of <pd, q> fused in its reduction
//   alpha = rr / <pd, q> ; z += alpha pd ; r -= alpha q ; partials of <r, r>
//   beta = rr_new / rr ; pd = r + beta pd
// Block preconditioners (Jacobi, the exact per-angle tridiagonal block, the
// exact per-block inverse) left the iteration count unchanged or raised it
// on this Gram (its conditioning comes from low-frequency modes shared by
// all blocks), so the iteration is unpreconditioned.
//
// Termination is decided on the device: the direction kernel sets a flag
// once ||r|| <= tol ||e|| and every later CG kernel returns at entry.  The
// host enqueues chunks of iterations ahead and reads the flag from pinned
// memory after a chunk completes, keeping the next chunk in flight, so the
// GPU does not idle on host round trips.  All dot products are two-stage
// fixed-order reductions, so runs are bitwise reproducible.
#include "pcg.h"

#include <algorithm>
#include <cmath>

namespace slim {

namespace {

constexpr int kThreads = 256;
constexpr int kChunk = 8;   // iterations enqueued per host check

enum { S_RR = 0, S_ALPHA, S_BETA, S_PQ, S_BB, S_COUNT };

__device__ __forceinline__ double block_sum(double v, double* sh) {
  for (int o = 32; o > 0; o >>= 1) v += __shfl_down(v, o, 64);
  const int w = threadIdx.x >> 6;
  if ((threadIdx.x & 63) == 0) sh[w] = v;
  __syncthreads();
  double r = 0.0;
  for (int q = 0; q < kThreads / 64; ++q) r += sh[q];
  __syncthreads();
  return r;
}

// Sum of a partial-sum array, computed redundantly by every workgroup in a
// fixed order (the same value in all of them).
__device__ __forceinline__ double sum_parts(const double* __restrict__ parts, int n, double* sh) {
  double a = 0.0;
  for (int k = threadIdx.x; k < n; k += kThreads) a += parts[k];
  return block_sum(a, sh);
}

// r = e, z = 0, pd = e; partials of <r, r>
__global__ __launch_bounds__(kThreads) void init_kernel(int p, int nres,
                                                        const double* __restrict__ res,
                                                        double* __restrict__ r,
                                                        double* __restrict__ z,
                                                        double* __restrict__ pd,
                                                        double* __restrict__ rr_parts) {
  __shared__ double sh[kThreads / 64];
  const int i = blockIdx.x * kThreads + threadIdx.x;
  double rr = 0.0;
  if (i < p) {
    const double e = (i >= p - nres) ? res[i - (p - nres)] : 0.0;
    r[i] = e;
    z[i] = 0.0;
    pd[i] = e;
    rr = e * e;
  }
  rr = block_sum(rr, sh);
  if (threadIdx.x == 0) rr_parts[blockIdx.x] = rr;
}

__global__ __launch_bounds__(kThreads) void init_scalars_kernel(const double* __restrict__ rr_parts,
                                                                int nparts, double* __restrict__ sc,
                                                                int* __restrict__ ctl) {
  __shared__ double sh[kThreads / 64];
  const double bb = sum_parts(rr_parts, nparts, sh);
  if (threadIdx.x == 0) {
    sc[S_RR] = bb;
    sc[S_BB] = bb;
    sc[S_BETA] = 0.0;
    ctl[kCtlDone] = (bb > 0.0) ? 0 : 1;
    ctl[kCtlIters] = 0;
  }
}

// alpha = rr / <pd, q>; z += alpha pd; r -= alpha q; partials of <r, r>
__global__ __launch_bounds__(kThreads) void update_kernel(int p, double* __restrict__ sc,
                                                          const double* __restrict__ pq_parts,
                                                          const double* __restrict__ pd,
                                                          const double* __restrict__ q,
                                                          double* __restrict__ z,
                                                          double* __restrict__ r,
                                                          double* __restrict__ rr_parts,
                                                          int nparts, const int* __restrict__ ctl) {
  if (ctl[kCtlDone]) return;
  __shared__ double sh[kThreads / 64];
  const int i = blockIdx.x * kThreads + threadIdx.x;
  const double pq = sum_parts(pq_parts, nparts, sh);
  const double alpha = (pq != 0.0) ? sc[S_RR] / pq : 0.0;
  if (blockIdx.x == 0 && threadIdx.x == 0) {
    sc[S_PQ] = pq;
    sc[S_ALPHA] = alpha;
  }
  double rr = 0.0;
  if (i < p) {
    z[i] = fma(alpha, pd[i], z[i]);
    const double rn = fma(-alpha, q[i], r[i]);
    r[i] = rn;
    rr = rn * rn;
  }
  rr = block_sum(rr, sh);
  if (threadIdx.x == 0) rr_parts[blockIdx.x] = rr;
}

// beta = rr_new / rr; pd = r + beta pd.  Every workgroup reads the current
// scalars in sc while workgroup 0 publishes the next ones in sc_next (the
// two sets alternate), counts the iteration and raises the stop flag.
__global__ __launch_bounds__(kThreads) void direction_kernel(int p, const double* __restrict__ sc,
                                                             double* __restrict__ sc_next,
                                                             const double* __restrict__ rr_parts,
                                                             int nparts, double tol2,
                                                             const double* __restrict__ r,
                                                             double* __restrict__ pd,
                                                             int* __restrict__ ctl) {
  if (ctl[kCtlDone]) return;
  __shared__ double sh[kThreads / 64];
  const double rr_new = sum_parts(rr_parts, nparts, sh);
  const double rr = sc[S_RR];
  const double beta = (rr != 0.0) ? rr_new / rr : 0.0;
  const int i = blockIdx.x * kThreads + threadIdx.x;
  if (i < p) pd[i] = fma(beta, pd[i], r[i]);
  if (blockIdx.x == 0 && threadIdx.x == 0) {
    sc_next[S_RR] = rr_new;
    sc_next[S_BETA] = beta;
    sc_next[S_BB] = sc[S_BB];
    ctl[kCtlIters] += 1;
    if (!(rr_new > tol2 * sc[S_BB])) ctl[kCtlDone] = 1;  // also stops on NaN
  }
}

}  // namespace

hipError_t pcg_alloc(PcgWork& w, int N, int64_t pmax) {
  hipError_t e;
  w.pmax = (int)pmax;
  w.nparts = (int)((pmax + kThreads - 1) / kThreads);
  const size_t np = (size_t)pmax * sizeof(double);
  if ((e = hipMalloc((void**)&w.r, np)) != hipSuccess) return e;
  if ((e = hipMalloc((void**)&w.pd, np)) != hipSuccess) return e;
  if ((e = hipMalloc((void**)&w.q, np)) != hipSuccess) return e;
  if ((e = hipMalloc((void**)&w.parts, (size_t)2 * w.nparts * sizeof(double))) != hipSuccess) return e;
  if ((e = hipMalloc((void**)&w.sc, 2 * S_COUNT * sizeof(double))) != hipSuccess) return e;
  if ((e = hipMalloc((void**)&w.ctl, kCtlCount * sizeof(int))) != hipSuccess) return e;
  if ((e = hipMalloc((void**)&w.u, (size_t)N * N * sizeof(float))) != hipSuccess) return e;
  if ((e = hipMalloc((void**)&w.uT, (size_t)N * N * sizeof(float))) != hipSuccess) return e;
  if ((e = hipHostMalloc((void**)&w.h_ctl, 2 * kCtlCount * sizeof(int), hipHostMallocDefault)) !=
      hipSuccess)
    return e;
  if ((e = hipHostMalloc((void**)&w.h_sc, 2 * S_COUNT * sizeof(double), hipHostMallocDefault)) !=
      hipSuccess)
    return e;
  for (int k = 0; k < 2; ++k)
    if ((e = hipEventCreateWithFlags(&w.ev[k], hipEventDisableTiming)) != hipSuccess) return e;
  return hipSuccess;
}

void pcg_free(PcgWork& w) {
  (void)hipFree(w.r);
  (void)hipFree(w.pd);
  (void)hipFree(w.q);
  (void)hipFree(w.parts);
  (void)hipFree(w.sc);
  (void)hipFree(w.ctl);
  (void)hipFree(w.u);
  (void)hipFree(w.uT);
  if (w.h_ctl) (void)hipHostFree(w.h_ctl);
  if (w.h_sc) (void)hipHostFree(w.h_sc);
  for (int k = 0; k < 2; ++k)
    if (w.ev[k]) (void)hipEventDestroy(w.ev[k]);
  w = PcgWork{};
}

hipError_t pcg_solve(PcgWork& w, const AngleGeom* geom, const AngleGeom* h_geom, float* partial,
                     int N, int R, const AngleList& win, double lam, const double* res, int nres,
                     double* z, double tol, int max_iter, int* iters, double* relres,
                     Profiler* prof, hipStream_t st) {
  const int p = win.n * R;
  const int nb = (p + kThreads - 1) / kThreads;
  double* pq_parts = w.parts;                      // written by the forward reduction
  double* rr_parts = w.parts + (size_t)w.nparts;  // written by init / update
  const double tol2 = tol * tol;
  hipError_t e;
  hipLaunchKernelGGL(init_kernel, dim3(nb), dim3(kThreads), 0, st, p, nres, res, w.r, z, w.pd,
                     rr_parts);
  hipLaunchKernelGGL(init_scalars_kernel, dim3(1), dim3(kThreads), 0, st, rr_parts, nb, w.sc,
                     w.ctl);
  if ((e = hipGetLastError()) != hipSuccess) return e;

  int enq = 0;     // iterations enqueued
  int chunks = 0;  // chunks enqueued
  int seen = 0;    // chunks whose flag copy has been read
  bool done = false;
  while (!done) {
    if (enq < max_iter) {
      const int todo = std::min(kChunk, max_iter - enq);
      for (int q = 0; q < todo; ++q, ++enq) {
        double* sc_cur = w.sc + (enq & 1) * S_COUNT;
        double* sc_nxt = w.sc + ((enq + 1) & 1) * S_COUNT;
        if (prof->on && (e = prof->begin(K_BACK, st)) != hipSuccess) return e;
        if ((e = launch_back(geom, N, R, win, nullptr, w.pd, w.u, nullptr, w.uT, nullptr, nullptr,
                             0, w.ctl, nullptr, nullptr, st)) != hipSuccess)
          return e;
        if (prof->on && (e = prof->end(st)) != hipSuccess) return e;
        if (prof->on && (e = prof->begin(K_FORWARD, st)) != hipSuccess) return e;
        if ((e = launch_forward(geom, h_geom, N, R, win, w.u, w.uT, 0, nullptr, 0, nullptr, w.q,
                                partial, w.pd, lam, pq_parts, w.ctl, st)) != hipSuccess)
          return e;
        if (prof->on && (e = prof->end(st)) != hipSuccess) return e;
        if (prof->on && (e = prof->begin(K_VEC, st)) != hipSuccess) return e;
        hipLaunchKernelGGL(update_kernel, dim3(nb), dim3(kThreads), 0, st, p, sc_cur, pq_parts,
                           w.pd, w.q, z, w.r, rr_parts, nb, w.ctl);
        hipLaunchKernelGGL(direction_kernel, dim3(nb), dim3(kThreads), 0, st, p, sc_cur, sc_nxt,
                           rr_parts, nb, tol2, w.r, w.pd, w.ctl);
        if ((e = hipGetLastError()) != hipSuccess) return e;
        if (prof->on && (e = prof->end(st)) != hipSuccess) return e;
      }
      int* slot = w.h_ctl + (chunks & 1) * kCtlCount;
      if ((e = hipMemcpyAsync(slot, w.ctl, kCtlCount * sizeof(int), hipMemcpyDeviceToHost, st)) !=
          hipSuccess)
        return e;
      if ((e = hipEventRecord(w.ev[chunks & 1], st)) != hipSuccess) return e;
      ++chunks;
    }
    // keep one chunk in flight while the previous one is checked
    if (chunks - seen >= 2 || enq >= max_iter) {
      if ((e = hipEventSynchronize(w.ev[seen & 1])) != hipSuccess) return e;
      const int* slot = w.h_ctl + (seen & 1) * kCtlCount;
      ++seen;
      if (slot[kCtlDone]) done = true;
      if (enq >= max_iter && seen == chunks) done = true;
    }
  }
  if ((e = hipStreamSynchronize(st)) != hipSuccess) return e;
  if (prof->on && (e = prof->harvest()) != hipSuccess) return e;
  int ctl[kCtlCount];
  if ((e = hipMemcpy(ctl, w.ctl, sizeof(ctl), hipMemcpyDeviceToHost)) != hipSuccess) return e;
  if ((e = hipMemcpy(w.h_sc, w.sc, 2 * S_COUNT * sizeof(double), hipMemcpyDeviceToHost)) !=
      hipSuccess)
    return e;
  const double* sc_last = w.h_sc + (ctl[kCtlIters] & 1) * S_COUNT;
  *iters = ctl[kCtlIters];
  const double bb = w.h_sc[S_BB];
  *relres = (bb > 0.0) ? std::sqrt(sc_last[S_RR] / bb) : 0.0;
  return hipSuccess;
}

}  // namespace slim
