// CG on the Gram system (lambda I + M M^T) z = [0; ...; 0; res]
// with matrix-free M (forward projector) and M^T (back-projector); used when
// p = rows(M) is too large for the explicit Gram.  Vectors in p-space are
// float64; the image-space intermediate M^T v is float32.  Scalars stay on
// the device; the host reads the residual norm every few iterations.
#pragma once

#include "slim_internal.h"

namespace slim {

struct PcgWork {
  int B = 0;                // slices
  int pmax = 0;             // rows of the largest window
  int nparts = 0;           // partial sums per slice
  double* r = nullptr;      // residuals          [B][pmax]
  double* pd = nullptr;     // search directions  [B][pmax]
  double* q = nullptr;      // G r                [B][pmax]
  double* s = nullptr;      // G pd (recurrence)  [B][pmax]
  double* parts = nullptr;  // per-workgroup partial dots <r,q>, <r,r>: [2][B][nparts]
  double* sc = nullptr;     // per-slice scalars, two sets used alternately [2][B][S]
  int* ctl = nullptr;       // per-slice stop flag and iteration count [B][kCtlCount]
  float* u = nullptr;       // M^T r              [B][N][N]
  float* uT = nullptr;      // its transpose      [B][N][N]
  int* h_ctl = nullptr;     // pinned host copy of ctl, written by the kernels [B][kCtlCount]
  int* d_live = nullptr;    // h_ctl's address on the device
  double* h_sc = nullptr;   // pinned copy of sc
  hipEvent_t ev[2] = {nullptr, nullptr};
  hipGraphExec_t graph_exec = nullptr;  // one chunk of iterations (graph mode)
  int last_iters = 0;       // iterations of the last solve reported (sizes the chunks)
};

// State of one CG solve, advanced by pcg_enqueue / pcg_poll so that several
// solves (contexts of different sizes) can be interleaved by one host loop.
// fa and ba point at win: a run must not be copied or moved once begun.
struct PcgRun {
  PcgWork* w = nullptr;
  AngleList win;
  FwdArgs fa;
  BackArgs ba;
  int p = 0, B = 0, nb = 0;
  double* z = nullptr;
  size_t z_stride = 0;
  double tol2 = 0.0;
  int max_iter = 0;
  Profiler* prof = nullptr;
  hipStream_t st = nullptr;
  int enq = 0;      // iterations enqueued
  int chunks = 0;   // chunks enqueued
  int seen = 0;     // chunks whose flag copy has been read
  bool graph_ready = false;  // graph_exec holds this run's chunk
  bool done = false;
};

hipError_t pcg_alloc(PcgWork& w, int N, int B, int64_t pmax);
void pcg_free(PcgWork& w);
// Solve the B systems (lambda I + M M^T) z_b = [0; res_b] (res_b: nres entries
// at res + b * res_stride), z_b at z + b * z_stride, all slices advancing
// together.  *iters and *relres: the largest over the slices.
// h_geom: host geometry table; partial: forward-projector workspace.
// use_graph: replay each chunk of iterations as one graph launch (needs a
// stream other than the null stream; chunks run eagerly while profiling).
hipError_t pcg_solve(PcgWork& w, const AngleGeom* geom, const AngleGeom* h_geom, float* partial,
                     int N, int R, int B, const AngleList& win, const ProjTune& tune, double lam,
                     const double* res, size_t res_stride, int nres, double* z, size_t z_stride,
                     double tol, int max_iter, bool use_graph, int* iters, double* relres,
                     Profiler* prof, hipStream_t st);

// The same solve in steps: begin enqueues the initialisation; enqueue adds
// the next chunk of iterations when fewer than two are in flight; poll reads
// the oldest chunk's stop flags once two are in flight (or the cap is
// reached) and sets run.done; finish_async enqueues the copy of the final
// scalars to pinned memory, which report reads (with the control words the
// kernels keep in pinned memory) once the caller has synchronised the
// stream.
hipError_t pcg_begin(PcgRun& run, PcgWork& w, const AngleGeom* geom, const AngleGeom* h_geom,
                     float* partial, int N, int R, int B, const AngleList& win,
                     const ProjTune& tune, double lam, const double* res, size_t res_stride,
                     int nres, double* z, size_t z_stride, double tol, int max_iter,
                     Profiler* prof, hipStream_t st);
hipError_t pcg_enqueue(PcgRun& run, bool use_graph);
hipError_t pcg_poll(PcgRun& run);
hipError_t pcg_finish_async(PcgRun& run);
void pcg_report(PcgRun& run, int* iters, double* relres);

// Grouped CG: the solves of several contexts (images of different sizes,
// the same window of angles) advanced in the same launches -- per iteration
// one grouped back-projection, one grouped forward (band kernel and
// reduction) and one grouped vector kernel over all contexts' slices, every
// workgroup finding its context in a descriptor table in device memory --
// with chunks of iterations replayed as one graph on one stream.  Each
// context keeps its own workspace, stop flags and iteration count (a
// converged slice's blocks return at entry); the runs come from pcg_begin.
constexpr int kMaxGroup = 16;

struct PcgGroupWork {
  int cap = 0;                 // contexts the descriptor tables hold
  size_t bytes = 0;
  void* h_desc = nullptr;      // pinned staging of the tables
  void* d_desc = nullptr;      // device tables
  hipEvent_t ev[2] = {nullptr, nullptr};
  hipGraphExec_t graph_exec = nullptr;
};

struct PcgGroupRun {
  PcgGroupWork* w = nullptr;
  PcgRun* runs[kMaxGroup] = {};
  int n = 0;
  GroupShape shape;
  int vec_total = 0;
  hipStream_t st = nullptr;
  int max_iter = 0, last_iters = 0;
  int enq = 0, chunks = 0, seen = 0;
  bool graph_ready = false;
  bool done = false;
};

hipError_t pcg_group_alloc(PcgGroupWork& gw, int n);
void pcg_group_free(PcgGroupWork& gw);
// The runs must have been begun (pcg_begin) with work ordered before st.
hipError_t pcg_group_begin(PcgGroupRun& gr, PcgGroupWork& gw, PcgRun* const* runs, int n,
                           hipStream_t st);
hipError_t pcg_group_enqueue(PcgGroupRun& gr, bool use_graph);
hipError_t pcg_group_poll(PcgGroupRun& gr);

}  // namespace slim
