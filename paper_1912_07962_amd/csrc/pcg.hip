// Conjugate gradients on the Gram system (lambda I + M M^T) z = e,
// e = [0; ...; 0; res], for a batch of slices that share M (each slice runs
// its own CG; all advance together in the same launches), with matrix-free
// M and M^T.
// The iteration is CG in the form with one reduction phase per iteration
// (Chronopoulos and Gear, 1989): the operator is applied to the residual and
// G pd is carried by a recurrence, so both dot products come from the same
// vectors and are formed together.  Per iteration:
//   u = M^T r                  back-projector (float32 image and transpose)
//   q = M u + lambda r         forward projector, float64 sums, with the
//                              partial sums of delta = <r, q> and
//                              gamma = <r, r> fused in its reduction
//   stop if gamma <= tol^2 <e, e>; else beta = gamma / gamma_old,
//   alpha = gamma / (delta - beta gamma / alpha_old) (first: beta = 0,
//   alpha = gamma / delta), pd = r + beta pd, s = q + beta s,
//   z += alpha pd, r -= alpha s
// (in exact arithmetic the iterates of standard CG).
// Block preconditioners (Jacobi, the exact per-angle tridiagonal block, the
// exact per-block inverse) left the iteration count unchanged or raised it
// on this Gram (its conditioning comes from low-frequency modes shared by
// all blocks), so the iteration is unpreconditioned.
//
// Termination is decided on the device: the vector kernel sets a slice's
// flag once its ||r|| <= tol ||e|| and every later CG kernel skips that
// slice (the projectors skip a slice tile once all its slices stopped).  The
// host enqueues chunks of iterations ahead and reads the flag after a chunk
// completes, keeping the next chunk in flight, so the GPU does not idle on
// host round trips.  The kernels that change the control word also write it
// to pinned host memory (mapped into the device's address space), so a
// chunk needs no copy: its completion event makes the words visible.  Chunks are 8 iterations (one graph
// launch) until a few iterations before the count of the previous solve on
// the same workspace, then 2, so that few iterations are enqueued past the
// stop; the first chunk of a solve is launched directly and the graph for
// the solve's window is captured while it runs.  All dot products are two-stage
// fixed-order reductions, so runs are bitwise reproducible.
#include "pcg.h"

#include <algorithm>
#include <cmath>
#include <vector>

namespace slim {

namespace {

constexpr int kThreads = 256;
constexpr int kChunk = 8;     // iterations per graph launch (host check)
constexpr int kTail = 2;      // iterations per host check near the predicted end
constexpr int kTailLead = 3;  // short chunks start this many iterations before it

// per-slice scalars: gamma and alpha of the last update (gamma 0 before the
// first), beta, <e, e>, and (set 0 only) the latest gamma
enum { S_RR = 0, S_ALPHA, S_BETA, S_BB, S_LAST, S_COUNT };

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

// Two block sums at once (a fixed order: the same values in every lane).
__device__ __forceinline__ void block_sum2(double& a, double& b, double* sh) {
  for (int o = 32; o > 0; o >>= 1) {
    a += __shfl_down(a, o, 64);
    b += __shfl_down(b, o, 64);
  }
  const int w = threadIdx.x >> 6;
  if ((threadIdx.x & 63) == 0) {
    sh[w] = a;
    sh[kThreads / 64 + w] = b;
  }
  __syncthreads();
  a = 0.0;
  b = 0.0;
  for (int q = 0; q < kThreads / 64; ++q) {
    a += sh[q];
    b += sh[kThreads / 64 + q];
  }
  __syncthreads();
}

// Sum of a partial-sum array, computed redundantly by every workgroup in a
// fixed order (the same value in all of them).
__device__ __forceinline__ double sum_parts(const double* __restrict__ parts, int n, double* sh) {
  double a = 0.0;
  for (int k = threadIdx.x; k < n; k += kThreads) a += parts[k];
  return block_sum(a, sh);
}

// r = e, z = 0, pd = 0, s = 0; partials of <r, r>.  blockIdx.y = slice.
__global__ __launch_bounds__(kThreads) void init_kernel(int p, int nres, int pmax, int nparts,
                                                        const double* __restrict__ res,
                                                        size_t res_stride,
                                                        double* __restrict__ r,
                                                        double* __restrict__ z, size_t z_stride,
                                                        double* __restrict__ pd,
                                                        double* __restrict__ sv,
                                                        double* __restrict__ rr_parts) {
  __shared__ double sh[kThreads / 64];
  const int sl = blockIdx.y;
  const int i = blockIdx.x * kThreads + threadIdx.x;
  const size_t vo = (size_t)sl * pmax;
  double rr = 0.0;
  if (i < p) {
    const double e = (i >= p - nres) ? res[(size_t)sl * res_stride + i - (p - nres)] : 0.0;
    r[vo + i] = e;
    z[(size_t)sl * z_stride + i] = 0.0;
    pd[vo + i] = 0.0;
    sv[vo + i] = 0.0;
    rr = e * e;
  }
  rr = block_sum(rr, sh);
  if (threadIdx.x == 0) rr_parts[(size_t)sl * nparts + blockIdx.x] = rr;
}

__global__ __launch_bounds__(kThreads) void init_scalars_kernel(const double* __restrict__ rr_parts,
                                                                int nb, int nparts,
                                                                double* __restrict__ sc,
                                                                int* __restrict__ ctl,
                                                                int* __restrict__ live) {
  __shared__ double sh[kThreads / 64];
  const int sl = blockIdx.y;
  const double bb = sum_parts(rr_parts + (size_t)sl * nparts, nb, sh);
  if (threadIdx.x == 0) {
    double* c = sc + (size_t)sl * S_COUNT;
    c[S_RR] = 0.0;   // no update yet: the first one takes beta = 0
    c[S_ALPHA] = 1.0;
    c[S_BB] = bb;
    c[S_BETA] = 0.0;
    c[S_LAST] = bb;
    const int done = (bb > 0.0) ? 0 : 1;
    ctl[sl * kCtlCount + kCtlDone] = done;
    ctl[sl * kCtlCount + kCtlIters] = 0;
    live[sl * kCtlCount + kCtlDone] = done;
    live[sl * kCtlCount + kCtlIters] = 0;
  }
}

// One update from the forward reduction's partials of delta = <r, q> and
// gamma = <r, r> (q = G r), each summed in a fixed order by every workgroup.
// Converged (gamma <= tol^2 <e, e>, NaN included): no update, workgroup 0
// raises the stop flag.  Otherwise pd = r + beta pd, s = q + beta s,
// z += alpha pd, r -= alpha s, and workgroup 0 publishes gamma and alpha in
// sc_next (the two sets alternate) and counts the iteration.  last: set 0 of
// the scalars (its S_LAST slot, read by no kernel, holds the latest gamma).
// (block bx of slice sl; shared by the one-context and the grouped launch)
__device__ __forceinline__ void cg_vector_body(int bx, int sl, int p, int pmax, int nb, int nparts,
                                               const double* __restrict__ sc_all,
                                               double* __restrict__ sc_next_all,
                                               double* __restrict__ last_all,
                                               const double* __restrict__ dq_parts,
                                               const double* __restrict__ rr_parts, double tol2,
                                               const double* __restrict__ q,
                                               double* __restrict__ r, double* __restrict__ pd,
                                               double* __restrict__ sv, double* __restrict__ z,
                                               size_t z_stride, int* __restrict__ ctl,
                                               int* __restrict__ live) {
  __shared__ double sh[2 * (kThreads / 64)];
  __shared__ int stop_sh;
  // every load of the workgroup (stop flag, scalars, partial dots, the
  // lane's vector entries) is issued before the first wait; a stopped
  // slice's workgroups read and leave without writing.  The stop flag is
  // read once per workgroup and shared through LDS: the slice's first
  // workgroup may set it during this launch, and waves reading it apart
  // could disagree (a wave leaving early would leave its slot of the block
  // sum unwritten for the waves that stay).
  if (threadIdx.x == 0) stop_sh = ctl[sl * kCtlCount + kCtlDone];
  const double* sc = sc_all + (size_t)sl * S_COUNT;
  const double bb = sc[S_BB], g_old = sc[S_RR], a_old = sc[S_ALPHA];
  const int i = bx * kThreads + threadIdx.x;
  const size_t o = (size_t)sl * pmax + min(i, p - 1);
  double* zs = z + (size_t)sl * z_stride;
  const double pd_o = pd[o], r_o = r[o], sv_o = sv[o], q_o = q[o];
  const double z_o = zs[min(i, p - 1)];
  double delta = 0.0, gamma = 0.0;
  for (int k = threadIdx.x; k < nb; k += kThreads) {
    delta += dq_parts[(size_t)sl * nparts + k];
    gamma += rr_parts[(size_t)sl * nparts + k];
  }
  block_sum2(delta, gamma, sh);   // its barriers publish stop_sh
  if (stop_sh) return;
  const bool conv = !(gamma > tol2 * bb);
  const double beta = (g_old > 0.0) ? gamma / g_old : 0.0;
  const double alpha = (g_old > 0.0) ? gamma / (delta - beta * gamma / a_old) : gamma / delta;
  if (bx == 0 && threadIdx.x == 0) {
    last_all[(size_t)sl * S_COUNT + S_LAST] = gamma;
    if (conv) {
      ctl[sl * kCtlCount + kCtlDone] = 1;
      live[sl * kCtlCount + kCtlDone] = 1;
    } else {
      double* sn = sc_next_all + (size_t)sl * S_COUNT;
      sn[S_RR] = gamma;
      sn[S_ALPHA] = alpha;
      sn[S_BETA] = beta;
      sn[S_BB] = bb;
      const int it = ctl[sl * kCtlCount + kCtlIters] + 1;
      ctl[sl * kCtlCount + kCtlIters] = it;
      live[sl * kCtlCount + kCtlIters] = it;
    }
  }
  if (conv) return;
  if (i < p) {
    const double pn = fma(beta, pd_o, r_o);
    const double sn = fma(beta, sv_o, q_o);
    pd[o] = pn;
    sv[o] = sn;
    zs[i] = fma(alpha, pn, z_o);
    r[o] = fma(-alpha, sn, r_o);
  }
}

__global__ __launch_bounds__(kThreads) void cg_vector_kernel(int p, int pmax, int nb, int nparts,
                                                             const double* __restrict__ sc_all,
                                                             double* __restrict__ sc_next_all,
                                                             double* __restrict__ last_all,
                                                             const double* __restrict__ dq_parts,
                                                             const double* __restrict__ rr_parts,
                                                             double tol2,
                                                             const double* __restrict__ q,
                                                             double* __restrict__ r,
                                                             double* __restrict__ pd,
                                                             double* __restrict__ sv,
                                                             double* __restrict__ z,
                                                             size_t z_stride,
                                                             int* __restrict__ ctl,
                                                             int* __restrict__ live) {
  cg_vector_body(blockIdx.x, blockIdx.y, p, pmax, nb, nparts, sc_all, sc_next_all, last_all,
                 dq_parts, rr_parts, tol2, q, r, pd, sv, z, z_stride, ctl, live);
}

// One context of a grouped vector launch (device memory): its CG workspace
// and the first workgroup of its nb x B blocks in the launch.
struct VecGroupDesc {
  double* sc;      // both scalar sets [2][B][S_COUNT]
  const double* q;
  double* r;
  double* pd;
  double* sv;
  double* z;
  const double* dq_parts;
  const double* rr_parts;
  int* ctl;
  int* live;
  size_t z_stride;
  double tol2;
  int p, pmax, nb, nparts, B, start;
};

// parity: the iteration's parity, which picks the current scalar set
__global__ __launch_bounds__(kThreads) void cg_vector_grouped(const VecGroupDesc* __restrict__ d,
                                                              int n, int parity) {
  const int w = blockIdx.x;
  int g = 0;
  while (g + 1 < n && w >= d[g + 1].start) ++g;
  const VecGroupDesc& a = d[g];
  const int lw = w - a.start;
  const size_t set = (size_t)a.B * S_COUNT;
  cg_vector_body(lw % a.nb, lw / a.nb, a.p, a.pmax, a.nb, a.nparts, a.sc + (parity & 1) * set,
                 a.sc + ((parity + 1) & 1) * set, a.sc, a.dq_parts, a.rr_parts, a.tol2, a.q, a.r,
                 a.pd, a.sv, a.z, a.z_stride, a.ctl, a.live);
}

}  // namespace

hipError_t pcg_alloc(PcgWork& w, int N, int B, int64_t pmax) {
  hipError_t e;
  w.B = B;
  w.pmax = (int)pmax;
  w.nparts = (int)((pmax + kThreads - 1) / kThreads);
  const size_t np = (size_t)B * pmax * sizeof(double);
  if ((e = hipMalloc((void**)&w.r, np)) != hipSuccess) return e;
  if ((e = hipMalloc((void**)&w.pd, np)) != hipSuccess) return e;
  if ((e = hipMalloc((void**)&w.q, np)) != hipSuccess) return e;
  if ((e = hipMalloc((void**)&w.s, np)) != hipSuccess) return e;
  if ((e = hipMalloc((void**)&w.parts, (size_t)2 * B * w.nparts * sizeof(double))) != hipSuccess)
    return e;
  if ((e = hipMalloc((void**)&w.sc, (size_t)2 * B * S_COUNT * sizeof(double))) != hipSuccess) return e;
  if ((e = hipMalloc((void**)&w.ctl, (size_t)B * kCtlCount * sizeof(int))) != hipSuccess) return e;
  if ((e = hipMalloc((void**)&w.u, (size_t)B * N * N * sizeof(float))) != hipSuccess) return e;
  if ((e = hipMalloc((void**)&w.uT, (size_t)B * N * N * sizeof(float))) != hipSuccess) return e;
  if ((e = hipHostMalloc((void**)&w.h_ctl, (size_t)B * kCtlCount * sizeof(int),
                         hipHostMallocMapped | hipHostMallocCoherent)) != hipSuccess)
    return e;
  if ((e = hipHostGetDevicePointer((void**)&w.d_live, w.h_ctl, 0)) != hipSuccess) return e;
  if ((e = hipHostMalloc((void**)&w.h_sc, (size_t)2 * B * S_COUNT * sizeof(double),
                         hipHostMallocDefault)) != hipSuccess)
    return e;
  for (int k = 0; k < 2; ++k)
    if ((e = hipEventCreateWithFlags(&w.ev[k], hipEventDisableTiming)) != hipSuccess) return e;
  return hipSuccess;
}

void pcg_free(PcgWork& w) {
  if (w.graph_exec) (void)hipGraphExecDestroy(w.graph_exec);
  w.graph_exec = nullptr;
  (void)hipFree(w.r);
  (void)hipFree(w.pd);
  (void)hipFree(w.q);
  (void)hipFree(w.s);
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

hipError_t pcg_begin(PcgRun& run, PcgWork& w, const AngleGeom* geom, const AngleGeom* h_geom,
                     float* partial, int N, int R, int B, const AngleList& win,
                     const ProjTune& tune, double lam, const double* res, size_t res_stride,
                     int nres, double* z, size_t z_stride, double tol, int max_iter,
                     Profiler* prof, hipStream_t st) {
  run.w = &w;
  run.win = win;
  run.p = win.n * R;
  run.B = B;
  run.nb = (run.p + kThreads - 1) / kThreads;
  run.z = z;
  run.z_stride = z_stride;
  run.tol2 = tol * tol;
  run.max_iter = max_iter;
  run.prof = prof;
  run.st = st;
  run.enq = run.chunks = run.seen = 0;
  run.done = false;
  run.graph_ready = false;
  const int np = w.nparts;
  double* rr_parts = w.parts + (size_t)B * np;  // written by init / the forward reduction
  const size_t img = (size_t)N * N;
  hipLaunchKernelGGL(init_kernel, dim3(run.nb, B), dim3(kThreads), 0, st, run.p, nres, w.pmax,
                     np, res, res_stride, w.r, z, z_stride, w.pd, w.s, rr_parts);
  hipLaunchKernelGGL(init_scalars_kernel, dim3(1, B), dim3(kThreads), 0, st, rr_parts, run.nb,
                     np, w.sc, w.ctl, w.d_live);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;

  BackArgs& ba = run.ba;
  ba = BackArgs();
  ba.tune = tune;
  ba.geom = geom;
  ba.N = N;
  ba.R = R;
  ba.B = B;
  ba.ids = &run.win;
  ba.v64 = w.r;
  ba.v_stride = w.pmax;
  ba.out = w.u;
  ba.xT = w.uT;
  ba.img_stride = img;
  ba.mode = 0;
  ba.stop = w.ctl;
  ba.stop_stride = kCtlCount;
  FwdArgs& fa = run.fa;
  fa = FwdArgs();
  fa.tune = tune;
  fa.geom = geom;
  fa.h_geom = h_geom;
  fa.N = N;
  fa.R = R;
  fa.B = B;
  fa.ids = &run.win;
  fa.img = w.u;
  fa.imgT = w.uT;
  fa.img_stride = img;
  fa.out64 = w.q;
  fa.out_stride = w.pmax;
  fa.partial = partial;
  fa.pd = w.r;
  fa.pd_stride = w.pmax;
  fa.lam = lam;
  fa.dots = w.parts;  // <r, q> partials
  fa.dots2 = rr_parts;  // <r, r> partials
  fa.dots_stride = np;
  fa.stop = w.ctl;
  fa.stop_stride = kCtlCount;
  return hipSuccess;
}

namespace {

// Enqueue CG iterations enq .. enq+todo-1 (kernels only).
hipError_t enqueue_iterations(PcgRun& run, int todo, bool timed) {
  PcgWork& w = *run.w;
  const int B = run.B, np = w.nparts;
  double* dq_parts = w.parts;
  double* rr_parts = w.parts + (size_t)B * np;
  Profiler* prof = run.prof;
  hipStream_t st = run.st;
  hipError_t e;
  for (int q = 0; q < todo; ++q) {
    const int it = run.enq + q;
    double* sc_cur = w.sc + (size_t)(it & 1) * B * S_COUNT;
    double* sc_nxt = w.sc + (size_t)((it + 1) & 1) * B * S_COUNT;
    if (timed && (e = prof->begin(K_BACK, st)) != hipSuccess) return e;
    if ((e = launch_back(run.ba, st)) != hipSuccess) return e;
    if (timed && (e = prof->end(st)) != hipSuccess) return e;
    // q = M u + lambda r and partials of <r, q>, <r, r>, fused into the
    // forward's reduction (timed inside: band kernel and reduction separately)
    run.fa.prof = timed ? prof : nullptr;
    if ((e = launch_forward(run.fa, st)) != hipSuccess) return e;
    if (timed && (e = prof->begin(K_VEC, st)) != hipSuccess) return e;
    hipLaunchKernelGGL(cg_vector_kernel, dim3(run.nb, B), dim3(kThreads), 0, st, run.p, w.pmax,
                       run.nb, np, sc_cur, sc_nxt, w.sc, dq_parts, rr_parts, run.tol2, w.q, w.r,
                       w.pd, w.s, run.z, run.z_stride, w.ctl, w.d_live);
    if ((e = hipGetLastError()) != hipSuccess) return e;
    if (timed && (e = prof->end(st)) != hipSuccess) return e;
  }
  return hipSuccess;
}

// The kernels of one full chunk as a graph (same arguments for every chunk
// of a solve: the window is fixed and the scalar sets alternate with the
// iteration's parity, which repeats every even-sized chunk).  An existing
// executable graph is updated in place when the kernels match, else rebuilt.
hipError_t chunk_graph(PcgRun& run) {
  PcgWork& w = *run.w;
  hipError_t e = hipStreamBeginCapture(run.st, hipStreamCaptureModeThreadLocal);
  if (e != hipSuccess) return e;
  hipError_t ek = enqueue_iterations(run, kChunk, false);
  hipGraph_t g = nullptr;
  e = hipStreamEndCapture(run.st, &g);
  if (ek != hipSuccess) {
    if (g) (void)hipGraphDestroy(g);
    return ek;
  }
  if (e != hipSuccess) return e;
  if (w.graph_exec) {
    hipGraphExecUpdateResult res;
    hipGraphNode_t bad = nullptr;
    if (hipGraphExecUpdate(w.graph_exec, g, &bad, &res) != hipSuccess ||
        res != hipGraphExecUpdateSuccess) {
      (void)hipGetLastError();
      (void)hipGraphExecDestroy(w.graph_exec);
      w.graph_exec = nullptr;
    }
  }
  if (!w.graph_exec) e = hipGraphInstantiate(&w.graph_exec, g, nullptr, nullptr, 0);
  (void)hipGraphDestroy(g);
  return e;
}

}  // namespace

hipError_t pcg_enqueue(PcgRun& run, bool use_graph) {
  if (run.done || run.enq >= run.max_iter || run.chunks - run.seen >= 2) return hipSuccess;
  PcgWork& w = *run.w;
  const int B = run.B;
  const int K = w.last_iters;
  const bool tail = K > 0 && run.enq + kChunk > K - kTailLead && run.enq < K + kChunk;
  const int todo = std::min(tail ? kTail : kChunk, run.max_iter - run.enq);
  hipError_t e;
  const bool timed = run.prof && run.prof->on;
  // graph chunks start at even iterations (the scalar sets alternate with
  // the parity); every chunk before is of even length
  if (use_graph && !timed && todo == kChunk && run.enq > 0 && (run.enq & 1) == 0) {
    if (!run.graph_ready) {
      if ((e = chunk_graph(run)) != hipSuccess) return e;
      run.graph_ready = true;
    }
    if ((e = hipGraphLaunch(w.graph_exec, run.st)) != hipSuccess) return e;
  } else {
    if ((e = enqueue_iterations(run, todo, timed)) != hipSuccess) return e;
  }
  run.enq += todo;
  if ((e = hipEventRecord(w.ev[run.chunks & 1], run.st)) != hipSuccess) return e;
  ++run.chunks;
  return hipSuccess;
}

hipError_t pcg_poll(PcgRun& run) {
  if (run.done) return hipSuccess;
  // keep one chunk in flight while the previous one is checked
  if (run.chunks - run.seen >= 2 || (run.enq >= run.max_iter && run.seen < run.chunks)) {
    PcgWork& w = *run.w;
    hipError_t e = hipEventSynchronize(w.ev[run.seen & 1]);
    if (e != hipSuccess) return e;
    // the control words as of this chunk's end or later (they only advance;
    // a later chunk may be writing them)
    const volatile int* live = w.h_ctl;
    ++run.seen;
    bool all = true;
    for (int b = 0; b < run.B; ++b) all = all && live[b * kCtlCount + kCtlDone] != 0;
    if (all || (run.enq >= run.max_iter && run.seen == run.chunks)) run.done = true;
  }
  return hipSuccess;
}

// ------------------------------------------------------------ grouped CG
static size_t vec_desc_offset(int n) { return (grouped_desc_bytes(n) + 255) & ~size_t(255); }

hipError_t pcg_group_alloc(PcgGroupWork& gw, int n) {
  pcg_group_free(gw);
  gw.cap = n;
  gw.bytes = vec_desc_offset(n) + (size_t)n * sizeof(VecGroupDesc);
  hipError_t e;
  if ((e = hipHostMalloc(&gw.h_desc, gw.bytes, hipHostMallocDefault)) != hipSuccess) return e;
  if ((e = hipMalloc(&gw.d_desc, gw.bytes)) != hipSuccess) return e;
  for (int k = 0; k < 2; ++k)
    if ((e = hipEventCreateWithFlags(&gw.ev[k], hipEventDisableTiming)) != hipSuccess) return e;
  return hipSuccess;
}

void pcg_group_free(PcgGroupWork& gw) {
  if (gw.graph_exec) (void)hipGraphExecDestroy(gw.graph_exec);
  if (gw.h_desc) (void)hipHostFree(gw.h_desc);
  (void)hipFree(gw.d_desc);
  for (int k = 0; k < 2; ++k)
    if (gw.ev[k]) (void)hipEventDestroy(gw.ev[k]);
  gw = PcgGroupWork{};
}

hipError_t pcg_group_begin(PcgGroupRun& gr, PcgGroupWork& gw, PcgRun* const* runs, int n,
                           hipStream_t st) {
  if (n < 1 || n > gw.cap || n > kMaxGroup) return hipErrorInvalidValue;
  gr.w = &gw;
  gr.n = n;
  gr.st = st;
  gr.enq = gr.chunks = gr.seen = 0;
  gr.done = false;
  gr.graph_ready = false;
  gr.max_iter = 0;
  gr.last_iters = 0;
  const FwdArgs* fa[kMaxGroup];
  const BackArgs* ba[kMaxGroup];
  for (int g = 0; g < n; ++g) {
    gr.runs[g] = runs[g];
    fa[g] = &runs[g]->fa;
    ba[g] = &runs[g]->ba;
    gr.max_iter = std::max(gr.max_iter, runs[g]->max_iter);
    gr.last_iters = std::max(gr.last_iters, runs[g]->w->last_iters);
  }
  hipError_t e = grouped_prepare(fa, ba, n, gw.h_desc, &gr.shape);
  if (e != hipSuccess) return e;
  VecGroupDesc* vd = reinterpret_cast<VecGroupDesc*>(static_cast<char*>(gw.h_desc) +
                                                     vec_desc_offset(n));
  gr.vec_total = 0;
  for (int g = 0; g < n; ++g) {
    const PcgRun& r = *runs[g];
    PcgWork& w = *r.w;
    VecGroupDesc& v = vd[g];
    v.sc = w.sc;
    v.q = w.q;
    v.r = w.r;
    v.pd = w.pd;
    v.sv = w.s;
    v.z = r.z;
    v.dq_parts = w.parts;
    v.rr_parts = w.parts + (size_t)r.B * w.nparts;
    v.ctl = w.ctl;
    v.live = w.d_live;
    v.z_stride = r.z_stride;
    v.tol2 = r.tol2;
    v.p = r.p;
    v.pmax = w.pmax;
    v.nb = r.nb;
    v.nparts = w.nparts;
    v.B = r.B;
    v.start = gr.vec_total;
    gr.vec_total += r.nb * r.B;
  }
  // the table reaches the device in the stream's order, before the first
  // chunk (a replayed graph reads the table as it is at replay time)
  return hipMemcpyAsync(gw.d_desc, gw.h_desc, gw.bytes, hipMemcpyHostToDevice, st);
}

namespace {

hipError_t group_iterations(PcgGroupRun& gr, int todo) {
  PcgGroupWork& gw = *gr.w;
  const VecGroupDesc* vd = reinterpret_cast<const VecGroupDesc*>(
      static_cast<const char*>(gw.d_desc) + vec_desc_offset(gr.n));
  hipError_t e;
  for (int q = 0; q < todo; ++q) {
    const int it = gr.enq + q;
    if ((e = launch_back_grouped(gw.d_desc, gr.shape, gr.st)) != hipSuccess) return e;
    if ((e = launch_forward_grouped(gw.d_desc, gr.shape, gr.st)) != hipSuccess) return e;
    hipLaunchKernelGGL(cg_vector_grouped, dim3(gr.vec_total), dim3(kThreads), 0, gr.st, vd, gr.n,
                       it & 1);
    if ((e = hipGetLastError()) != hipSuccess) return e;
  }
  return hipSuccess;
}

hipError_t group_chunk_graph(PcgGroupRun& gr) {
  PcgGroupWork& gw = *gr.w;
  hipError_t e = hipStreamBeginCapture(gr.st, hipStreamCaptureModeThreadLocal);
  if (e != hipSuccess) return e;
  hipError_t ek = group_iterations(gr, kChunk);
  hipGraph_t g = nullptr;
  e = hipStreamEndCapture(gr.st, &g);
  if (ek != hipSuccess) {
    if (g) (void)hipGraphDestroy(g);
    return ek;
  }
  if (e != hipSuccess) return e;
  if (gw.graph_exec) {
    hipGraphExecUpdateResult res;
    hipGraphNode_t bad = nullptr;
    if (hipGraphExecUpdate(gw.graph_exec, g, &bad, &res) != hipSuccess ||
        res != hipGraphExecUpdateSuccess) {
      (void)hipGetLastError();
      (void)hipGraphExecDestroy(gw.graph_exec);
      gw.graph_exec = nullptr;
    }
  }
  if (!gw.graph_exec) e = hipGraphInstantiate(&gw.graph_exec, g, nullptr, nullptr, 0);
  (void)hipGraphDestroy(g);
  return e;
}

}  // namespace

hipError_t pcg_group_enqueue(PcgGroupRun& gr, bool use_graph) {
  if (gr.done || gr.enq >= gr.max_iter || gr.chunks - gr.seen >= 2) return hipSuccess;
  PcgGroupWork& gw = *gr.w;
  const int K = gr.last_iters;
  const bool tail = K > 0 && gr.enq + kChunk > K - kTailLead && gr.enq < K + kChunk;
  const int todo = std::min(tail ? kTail : kChunk, gr.max_iter - gr.enq);
  hipError_t e;
  if (use_graph && gr.st != nullptr && todo == kChunk && gr.enq > 0 && (gr.enq & 1) == 0) {
    if (!gr.graph_ready) {
      if ((e = group_chunk_graph(gr)) != hipSuccess) return e;
      gr.graph_ready = true;
    }
    if ((e = hipGraphLaunch(gw.graph_exec, gr.st)) != hipSuccess) return e;
  } else {
    if ((e = group_iterations(gr, todo)) != hipSuccess) return e;
  }
  gr.enq += todo;
  if ((e = hipEventRecord(gw.ev[gr.chunks & 1], gr.st)) != hipSuccess) return e;
  ++gr.chunks;
  return hipSuccess;
}

hipError_t pcg_group_poll(PcgGroupRun& gr) {
  if (gr.done) return hipSuccess;
  if (gr.chunks - gr.seen >= 2 || (gr.enq >= gr.max_iter && gr.seen < gr.chunks)) {
    PcgGroupWork& gw = *gr.w;
    hipError_t e = hipEventSynchronize(gw.ev[gr.seen & 1]);
    if (e != hipSuccess) return e;
    ++gr.seen;
    bool all = true;
    for (int g = 0; g < gr.n; ++g) {
      const PcgRun& r = *gr.runs[g];
      const volatile int* live = r.w->h_ctl;
      for (int b = 0; b < r.B; ++b) all = all && live[b * kCtlCount + kCtlDone] != 0;
    }
    if (all || (gr.enq >= gr.max_iter && gr.seen == gr.chunks)) gr.done = true;
  }
  return hipSuccess;
}

hipError_t pcg_finish_async(PcgRun& run) {
  PcgWork& w = *run.w;
  return hipMemcpyAsync(w.h_sc, w.sc, (size_t)2 * run.B * S_COUNT * sizeof(double),
                        hipMemcpyDeviceToHost, run.st);
}

void pcg_report(PcgRun& run, int* iters, double* relres) {
  PcgWork& w = *run.w;
  const int B = run.B;
  const volatile int* ctl = w.h_ctl;   // final once the stream is synchronised
  int it_max = 0;
  double rel_max = 0.0;
  bool finite = true;
  for (int b = 0; b < B; ++b) {
    const int it = ctl[b * kCtlCount + kCtlIters];
    const double* s0 = w.h_sc + (size_t)b * S_COUNT;   // set 0: <e, e> and the latest gamma
    it_max = std::max(it_max, it);
    // a non-finite right-hand side (data or iterate) stops the CG at once
    finite = finite && std::isfinite(s0[S_BB]) && std::isfinite(s0[S_LAST]);
    if (s0[S_BB] > 0.0) rel_max = std::max(rel_max, std::sqrt(s0[S_LAST] / s0[S_BB]));
  }
  w.last_iters = it_max;
  *iters = it_max;
  *relres = finite ? rel_max : NAN;
}

hipError_t pcg_solve(PcgWork& w, const AngleGeom* geom, const AngleGeom* h_geom, float* partial,
                     int N, int R, int B, const AngleList& win, const ProjTune& tune, double lam,
                     const double* res, size_t res_stride, int nres, double* z, size_t z_stride,
                     double tol, int max_iter, bool use_graph, int* iters, double* relres,
                     Profiler* prof, hipStream_t st) {
  PcgRun run;
  hipError_t e = pcg_begin(run, w, geom, h_geom, partial, N, R, B, win, tune, lam, res,
                           res_stride, nres, z, z_stride, tol, max_iter, prof, st);
  if (e != hipSuccess) return e;
  while (!run.done) {
    if ((e = pcg_enqueue(run, use_graph)) != hipSuccess) return e;
    if ((e = pcg_poll(run)) != hipSuccess) return e;
  }
  if ((e = pcg_finish_async(run)) != hipSuccess) return e;
  if ((e = hipStreamSynchronize(st)) != hipSuccess) return e;
  if (prof && prof->on && (e = prof->harvest()) != hipSuccess) return e;
  pcg_report(run, iters, relres);
  return hipSuccess;
}

}  // namespace slim
