// Internal declarations of the 3D parallel-beam path: the per-direction
// geometry table and the launchers of its projectors and CG kernels.
#pragma once

#include "slim_internal.h"

namespace slim {

// Per-direction geometry.  Voxel (k, i, j) has centre ((j, i, k) - hN) h with
// hN = (N-1)/2; a ray (q, t) of the n_det x n_det detector is
// {(t - hn) h e_u + (q - hn) h e_v + tau w} with hn = (n_det-1)/2.  With m the
// major axis of w and a, b the other two, the ray crosses the plane of voxel
// index k along m at index coordinates (in voxels, along a and b)
//     f_a(k) = hN + (t - hn) La[0] + (q - hn) La[1] + (k - hN) sa,
// (f_b likewise), La = (e_u[a] - e_u[m] sa, e_v[a] - e_v[m] sa), sa = w_a/w_m.
// For a voxel c the displacement from its own ray's crossing point, in
// voxels, is (P - c)_a = La[0] du + La[1] dv with (du, dv) the detector
// offset (in pixels) of the ray from the voxel's projection
// (c.e_u / h + hn, c.e_v / h + hn); only |du| < |e_u[a]| + |e_u[b]| <= sqrt 2
// (dv likewise) can give a non-zero weight.
struct DirGeom {
  double eu[3], ev[3];   // detector basis
  double La[2], Lb[2];   // crossing-point displacement per detector pixel
  double sa, sb;         // crossing-point change per plane along m
  double scale;          // h / |w_m|
  double wu, wv;         // |e_u[a]| + |e_u[b]|, |e_v[a]| + |e_v[b]|: candidate half-widths
  int m, a, b;           // major axis, the other two (x = 0, y = 1, z = 2)
  int pad;
};

// Padded volume layouts read by the forward projector and written by the
// back-projector: stored with axis m slowest (plane along m, then the higher
// of the other two axes, then the lower), each row of N voxels preceded by
// kPad zeros and followed by zeros up to the pitch lay_pitch(N), a multiple
// of four (16-byte rows).  The pads are zeroed once and never written.
constexpr int kPad = 4;
__host__ __device__ inline int lay_pitch(int N) { return (N + 2 * kPad + 3) / 4 * 4; }
inline size_t lay_floats(int N) { return (size_t)N * N * lay_pitch(N); }

// Directions of one launch (a window of r+1 blocks of g directions).
struct DirList {
  int n;
  int id[kMaxList];
};

// Forward projection over the directions of ids (slot s = ids.id[s]):
//   v[s][q][t] = sum A[(ids[s],q,t), voxel] x[voxel]   (float64 ray sums)
// minus sub[ids[s]][q][t] when sub is given (the data, [n_dirs][n][n]),
// written to out64 / out32 [s][q][t].  CG tail when pd is given:
// out64 = v + lam pd, per-workgroup partial sums of pd . out64 into dots
// (fwd3_num_workgroups values, one per 256 outputs, fixed order).  Returns
// at entry when ctl[kCtlDone] is set.
// The volume is read in the padded layout of each direction's major axis
// m, lay[m]; only the layouts of the list's directions are read.
struct Fwd3Args {
  const DirGeom* geom = nullptr;
  DirList ids;
  int N = 0, n = 0;
  const float* lay[3] = {nullptr, nullptr, nullptr};
  const float* sub = nullptr;
  float* out32 = nullptr;
  double* out64 = nullptr;
  const double* pd = nullptr;
  double lam = 0.0;
  double* dots = nullptr;
  const int* ctl = nullptr;
  double* part = nullptr;   // workspace: fwd3_part_doubles(n, ids.n) doubles
};
hipError_t launch_fwd3(const Fwd3Args& a, hipStream_t st);
// Workgroups of the reduction (= the dot partials it writes) and the
// partial-sum workspace of a forward over n_ids directions.
int fwd3_num_workgroups(int n, int n_ids);
size_t fwd3_part_doubles(int n, int n_ids);

// Back-projection over the directions of ids, the exact adjoint of the
// forward: s[voxel] = sum_s sum_(q,t) A[(ids[s],q,t), voxel] v[s][q][t] with v
// float32 (v32) or float64 (v64), [s][q][t].  mode 0: out = s in the
// standard [z][y][x] layout when out is given, and lay[m] = s in the padded
// layout of major axis m for every m whose lay[m] is given.  mode 1:
// x -= s in place and per-workgroup float64 partial norms (||s||^2,
// ||x_new||^2, ||x_new - x_true||^2) into partials[wg * 3 + k]
// (back3_num_workgroups values).  Returns at entry when ctl[kCtlDone] is set.
struct Back3Args {
  const DirGeom* geom = nullptr;
  DirList ids;
  int N = 0, n = 0;
  const float* v32 = nullptr;
  const double* v64 = nullptr;
  float* out = nullptr;
  float* lay[3] = {nullptr, nullptr, nullptr};
  float* x = nullptr;
  const float* x_true = nullptr;
  double* partials = nullptr;
  int mode = 0;
  const int* ctl = nullptr;
};
hipError_t launch_back3(const Back3Args& a, hipStream_t st);
// dst = src (standard layout) in the padded layout of major axis m.
hipError_t launch_relayout3(const float* src, float* dst, int N, int m, hipStream_t st);
int64_t back3_num_workgroups(int N);

// float64 scalars of the CG, in its device buffer sc.
enum { SC3_RR = 0, SC3_RR0, SC3_ALPHA, SC3_TOL2, SC3_PQ, SC3_BETA, SC3_RY, SC3_COUNT };

// CG on (lam I + M M^T) z = e in float64 (e: p entries), matrix-free,
// preconditioned by minv (the inverse of the Gram diagonal, diag3) when minv
// is non-NULL, plain otherwise (y = r below):
//   init:  r = e, y = minv r, pd = y, z = 0, rr = rr0 = e.e, ry = r.y
//          (ctl done if e = 0)
//   iteration: u = M^T pd (back), q = M u + lam pd with partial dots
//   (forward tail), alpha = ry / pd.q, z += alpha pd, r -= alpha q,
//   rr' = r.r, ry' = r.(minv r), stop when rr' <= tol^2 rr0, else
//   pd = minv r + (ry'/ry) pd.
// sc holds the scalars; ctl [done, iterations, non-finite].  parts holds
// 2 cg3_num_parts(p) doubles.
hipError_t launch_diag3(const DirGeom* geom, const DirList& ids, int N, int n, double lam,
                        double* minv, hipStream_t st);
hipError_t launch_cg3_init(const double* e, const double* minv, double* r, double* pd, double* z,
                           int p, double* parts, int nparts_cap, double* sc, int* ctl, double tol2,
                           hipStream_t st);
hipError_t launch_cg3_alpha(const double* dots, int nd, double* sc, int* ctl, hipStream_t st);
hipError_t launch_cg3_update(double* z, double* r, const double* pd, const double* q,
                             const double* minv, int p, double* parts, double* sc, int* ctl,
                             hipStream_t st);
hipError_t launch_cg3_beta(double* r, const double* minv, double* pd, int p, const double* parts,
                           double* sc, int* ctl, hipStream_t st);
int cg3_num_parts(int p);

}  // namespace slim
