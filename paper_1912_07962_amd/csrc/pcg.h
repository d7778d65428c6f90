// CG on the Gram system (lambda I + M M^T) z = [0; ...; 0; res]
// with matrix-free M (forward projector) and M^T (back-projector); used when
// p = rows(M) is too large for the explicit Gram.  Vectors in p-space are
// float64; the image-space intermediate M^T v is float32.  Scalars stay on
// the device; the host reads the residual norm every few iterations.
#pragma once

#include "slim_internal.h"

namespace slim {

struct PcgWork {
  int pmax = 0;
  int nparts = 0;
  double* r = nullptr;      // residual           [pmax]
  double* pd = nullptr;     // search direction   [pmax]
  double* q = nullptr;      // G pd               [pmax]
  double* parts = nullptr;  // per-workgroup partial dots <pd,q>, <r,r> [2][nparts]
  double* sc = nullptr;     // device scalars, two sets used alternately
  int* ctl = nullptr;       // stop flag and iteration count
  float* u = nullptr;       // M^T pd             [N][N]
  float* uT = nullptr;      // its transpose      [N][N]
  int* h_ctl = nullptr;     // pinned copies of ctl, one per chunk in flight
  double* h_sc = nullptr;   // pinned copy of sc
  hipEvent_t ev[2] = {nullptr, nullptr};
};

hipError_t pcg_alloc(PcgWork& w, int N, int64_t pmax);
void pcg_free(PcgWork& w);
// Solve for one slice: rhs = [0; res] (res: last nres entries), z: [p] out.
// h_geom: host geometry table; partial: forward-projector workspace.
hipError_t pcg_solve(PcgWork& w, const AngleGeom* geom, const AngleGeom* h_geom, float* partial,
                     int N, int R, const AngleList& win, double lam, const double* res, int nres,
                     double* z, double tol, int max_iter, int* iters, double* relres,
                     Profiler* prof, hipStream_t st);

// dst = src^T (if dst), bf16 copies of src (bs) and src^T (bsT) if given.
hipError_t launch_transpose(const float* src, float* dst, int N, uint16_t* bs, uint16_t* bsT,
                            hipStream_t st);

}  // namespace slim
