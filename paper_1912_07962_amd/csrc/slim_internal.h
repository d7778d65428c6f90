// Internal declarations of the slimLS library: context, geometry table,
// the shared Joseph weight evaluation, and the kernel launchers.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include <string>
#include <vector>

#include "../../include/slim.h"

namespace slim {

// Largest number of angles a single launch walks (window of r+1 blocks of g
// angles).  Angle lists travel by value in the kernel arguments.
constexpr int kMaxList = 256;

struct AngleList {
  int n;
  int id[kMaxList];
};

// Per-angle geometry.  The detector coordinate of pixel (i, j) for an angle
// is t = jj*c + ii*s + off in units of the ray spacing, with jj = j-(N-1)/2,
// ii = i-(N-1)/2, off = (R-1)/2.  Rays of "row-major" angles (|c| >= |s|)
// cross every image row once; the others cross every column once.
struct AngleGeom {
  double c, s;      // cos(theta), sin(theta)
  float hd;         // h / d,  d = max(|c|, |s|)
  float invd;       // 1 / d
  int colmajor;     // 1 if |s| > |c|
  int pad;
  // Forward-projector constants of the angle's own orientation (filled by
  // fwd_angle_consts for the image size N and detector size R): ray t is at
  // position p(k) = fma(t, f_inv, f_c0) + k f_n1 in the row (column) k it
  // crosses, in pixels counted from the start of the projector's padded band
  // row; f_S is f_n1 in 32.32 fixed point; for f_n1 != 0 the rows whose
  // position lies within half a pixel beyond the image's border pixels are
  // those between fma(t, f_qs, f_qa) and fma(t, f_qs, f_qb).
  double f_inv, f_c0, f_n1, f_qa, f_qb, f_qs;
  long long f_S;
};
void fwd_angle_consts(AngleGeom& g, int N, int R);

// Canonical detector coordinate of a pixel.  The Gram kernel evaluates
// exactly this expression; the back-projector evaluates it at each tile's
// first pixel and reaches the tile's other pixels by row and column steps in
// 32.32 fixed point (within 1e-8 pixel), and the forward projector evaluates
// the same closed form along rays, so all three agree up to float32 weight
// rounding.
__device__ __forceinline__ double det_coord(double s, double c, double ii, double jj, double off) {
  return fma(jj, c, fma(ii, s, off));
}
__device__ __forceinline__ double det_coord(const AngleGeom& g, double ii, double jj, double off) {
  return det_coord(g.s, g.c, ii, jj, off);
}

// Joseph weight of a pixel at detector coordinate t on ray tr, 0 if tr is
// neither floor(t) nor floor(t)+1 (those two are the only rays that can be
// within d of t, since d <= 1).
__device__ __forceinline__ float ray_weight(const AngleGeom& g, double t, int tr) {
  const double fl = floor(t);
  const int t0 = (int)fl;
  const double f = t - fl;  // exact
  float dist;
  if (t0 == tr) dist = (float)f;
  else if (t0 + 1 == tr) dist = (float)(1.0 - f);
  else return 0.f;
  return g.hd * fmaxf(0.f, 1.f - dist * g.invd);
}

// Both non-zero candidates of a pixel: rays t0 and t0+1 with weights w0, w1.
__device__ __forceinline__ void pixel_weights(const AngleGeom& g, double t, int& t0, float& w0,
                                              float& w1) {
  const double fl = floor(t);
  t0 = (int)fl;
  const double f = t - fl;
  w0 = g.hd * fmaxf(0.f, 1.f - (float)f * g.invd);
  w1 = g.hd * fmaxf(0.f, 1.f - (float)(1.0 - f) * g.invd);
}

// Device-side CG control word: stop flag and iteration count.  Kernels that
// take a `stop` pointer return at entry when stop[kCtlDone] is set.
constexpr int kCtlDone = 0, kCtlIters = 1, kCtlCount = 2;

// Optional per-kernel timing with HIP events on the launch stream.  Kinds:
enum KernelKind { K_FORWARD = 0, K_BACK, K_GRAM, K_CHOL, K_VEC, K_RESID, K_UPDATE, K_FWD_REDUCE, K_COUNT };

struct Profiler {
  bool on = false;
  std::vector<hipEvent_t> pool;
  std::vector<int> kind;   // kind of each recorded pair
  int used = 0;            // pairs recorded since the last harvest
  double total_ms[K_COUNT] = {};
  long long launches[K_COUNT] = {};
  hipError_t begin(int k, hipStream_t st);
  hipError_t end(hipStream_t st);
  hipError_t harvest();  // stream must be synchronised
  void release();
};

// ---- launchers (return hipError_t of the launch) --------------------------
// Slice tile of the batched projectors (1, 2 or 4 slices per workgroup).
int slice_tile(int B);

// Forward projection of B slices sharing the geometry:
//   out[slice][a][t] = sum_pix A[(ids[a],t),pix] img[slice][pix] - sub[slice][ids[a]][t]
// accumulated in float64 per ray, written as float (out32) and/or double (out64).
// img (float32, or bf16 bit patterns when img_bf16) is required; imgT, its
// transpose in the same format, is optional: column-stepping angles walk
// bands of imgT's rows when it is given, else bands of img's columns
// (transposed while staged).  sub likewise with sub_bf16.  Strides are in
// elements.
// partial: workspace of forward_partial_floats(...) floats.  CG tail when pd
// is non-NULL: out += lam * pd and per-workgroup partial sums of pd . out into
// dots[slice * dots_stride + w], one per 256 outputs w (and of pd . pd into
// dots2 likewise, when dots2 is non-NULL).  Slices whose
// stop[slice * stop_stride + kCtlDone] is set are skipped.
// Launch shape of the projectors; zero fields take the built-in rules (the
// autotuner measures and fills them).
struct ProjTune {
  int fwd_bt = 0;     // forward slice tile: 1, 2 or 4
  int fwd_items = 0;  // cap on rays per lane of the forward
  int fwd_slots = 0;  // resident forward workgroups per CU the grid aims at
  int back_bt = 0;    // back-projector slice tile: 1, 2 or 4
};

struct FwdArgs {
  ProjTune tune;
  Profiler* prof = nullptr;   // when set (and on): events around the band kernel (K_FORWARD)
                              // and the reduction (K_FWD_REDUCE)
  const AngleGeom* geom = nullptr;
  const AngleGeom* h_geom = nullptr;   // host copy (the launch plan groups angles)
  int N = 0, R = 0, B = 1;
  const AngleList* ids = nullptr;
  const void* img = nullptr;
  const void* imgT = nullptr;
  size_t img_stride = 0;
  int img_bf16 = 0;
  const void* sub = nullptr;
  size_t sub_stride = 0;
  int sub_bf16 = 0;
  float* out32 = nullptr;
  double* out64 = nullptr;
  size_t out_stride = 0;
  float* partial = nullptr;
  const double* pd = nullptr;
  size_t pd_stride = 0;
  double lam = 0.0;
  double* dots = nullptr;
  double* dots2 = nullptr;
  size_t dots_stride = 0;
  const int* stop = nullptr;
  int stop_stride = 0;
};
hipError_t launch_forward(const FwdArgs& a, hipStream_t st);
// Largest rays-per-lane cap the forward supports for slice tile bt.
int forward_max_items(int bt);
size_t forward_partial_floats(const AngleGeom* h_geom, int N, int R, const AngleList& ids, int B,
                              const ProjTune& tune);

// Back-projection of B slices: s[slice][pix] = sum_a sum_t A[(ids[a],t),pix] v[slice][a][t]
// with v float (v32) or double (v64).  mode 0: out = s (and out^T into xT).
// mode 1: s += shrink * x (the Tikhonov term of eq. (slimTik) with L = I;
// shrink = 0 otherwise), x -= s in place, optional transposed copy xT,
// optional bf16 copies xs, xsT (round to nearest even), and per-workgroup
// float64 partial norms (||s||^2, ||x_new||^2, ||x_new - x_true||^2) into
// partials[(slice * back_num_workgroups(N) + wg) * 3 + k].
struct BackArgs {
  ProjTune tune;
  const AngleGeom* geom = nullptr;
  int N = 0, R = 0, B = 1;
  const AngleList* ids = nullptr;
  const float* v32 = nullptr;
  const double* v64 = nullptr;
  size_t v_stride = 0;
  float* out = nullptr;
  float* x = nullptr;
  float* xT = nullptr;
  const float* x_true = nullptr;
  size_t img_stride = 0;
  double* partials = nullptr;
  int mode = 0;
  const int* stop = nullptr;
  int stop_stride = 0;
  uint16_t* xs = nullptr;
  uint16_t* xsT = nullptr;
  float shrink = 0.f;
};
hipError_t launch_back(const BackArgs& a, hipStream_t st);
int back_num_workgroups(int N);

// Grouped CG products: the work of several contexts (images of different
// sizes, the same angle list) in one launch per kernel -- one back-projector
// launch for u_g = M^T v_g, one band launch and one reduction launch for
// q_g = M u_g + lam pd_g with the dots -- every workgroup finding its
// context in a table of descriptors in device memory.  grouped_prepare
// fills host_desc (grouped_desc_bytes(n) bytes) from the contexts' CG
// arguments (BackArgs mode 0 with float64 v; FwdArgs with pd, float32
// images, no data) and returns the launch shape; the caller copies the table
// to device memory (dev_desc) before the launches, which take only its
// address (so a captured graph stays valid while the table is rewritten
// between replays).  The back-projector runs with the smallest slice tile
// of the contexts; every other launch shape is each context's own, so the
// results equal the one-context launches'.
struct GroupShape {
  int n = 0;
  int back_bt = 1;
  int back_total = 0;    // back-projector workgroups
  int band_total = 0;    // band-kernel positions
  int band_grid = 0;     // band-kernel grid: 8 x the contexts' positions per XCD
  size_t band_lds = 0;   // dynamic LDS of the band kernel (largest band)
  int red_total = 0;     // reduction workgroups
};
size_t grouped_desc_bytes(int n);
hipError_t grouped_prepare(const FwdArgs* const* fa, const BackArgs* const* ba, int n,
                           void* host_desc, GroupShape* shape);
hipError_t launch_back_grouped(const void* dev_desc, const GroupShape& shape, hipStream_t st);
hipError_t launch_forward_grouped(const void* dev_desc, const GroupShape& shape, hipStream_t st);

// Per slice, sum the n partial 3-vectors in a fixed order into out[3*slice..].// Per slice, sum the n partial 3-vectors in a fixed order into out[3*slice..].
hipError_t launch_reduce3(const double* partials, int n, int B, double* out, hipStream_t st);

// dst = src^T (if dst), bf16 copies of src (bs) and src^T (bsT) if given, for
// B slices with the given element stride.
hipError_t launch_transpose(const float* src, float* dst, int N, int B, size_t stride,
                            uint16_t* bs, uint16_t* bsT, hipStream_t st);

// Gram block: out[(a,t),(b,u)] = sum_pix A[(ida[a],t),pix] A[(idb[b],u),pix],
// float64, row-major with leading dimension ld.
hipError_t launch_gram(const AngleGeom* geom, int N, int R, const AngleList& ida,
                       const AngleList& idb, double* out, int64_t ld, hipStream_t st);

// Copy a tile (rows x cols, leading dimension lds) into G at (r0, c0) with
// leading dimension ldg, adding diag to its diagonal when add_diag != 0.
// The lower triangle of G (ldg) from the tiles of the W window positions in
// one launch: position P holds ring slot (first + P) mod S, tile (sp, sq) at
// tiles + (sp S + sq) ell^2 (row-major ell x ell), lambda added on the
// diagonal.  hipErrorInvalidValue if W (W + 1) / 2 or ell exceed 65535.
hipError_t launch_tile_assemble(const double* tiles, int S, int first, int W, int ell, double* G,
                                int64_t ldg, double lam, hipStream_t st);
hipError_t launch_tile_copy(const double* src, int64_t lds, double* G, int64_t ldg, int r0,
                            int c0, int rows, int cols, double diag, int add_diag,
                            hipStream_t st);

// Lower Cholesky of the p x p row-major matrix G (ld) in place.  info[0] is
// set to 1 + index of the first non-positive pivot (0 on success).  work
// (chol_work_doubles(p)) receives the inverses of the 64 x 64 diagonal
// blocks of L, which the triangular solves use.
inline size_t chol_work_doubles(int64_t p) { return (size_t)((p + 63) / 64) * 64 * 64; }
hipError_t launch_cholesky(double* G, int64_t ld, int p, int* info, double* work,
                           hipStream_t st);

// For each of B right-hand sides: solve L y = e with e = [0; rhs] (rhs: the
// last nr entries, rhs64 + slice * rhs_stride) and L^T z = y
// (z + slice * z_stride, float64 [p]).  ywork: B * z_stride doubles of
// scratch (y per right-hand side).
hipError_t launch_chol_solve(const double* L, int64_t ld, int p, int nr, const double* work,
                             const double* rhs64, size_t rhs_stride, double* z, size_t z_stride,
                             double* ywork, int B, hipStream_t st);

// out[s][i][t] = b[s][ids[i]][t] as float32 for B slices (b float32 or bf16,
// slice stride n_angles * R).
hipError_t launch_gather_rows(const void* b, int b_bf16, int n_angles, int R, int B,
                              const AngleList& ids, float* out, hipStream_t st);

// slimTik right-hand sides for B slices: rhs[j] = -c mx[j] for j < p, plus
// res[j - (p - nres)] for the last nres entries (eq. (slimTik), L = I).
hipError_t launch_tik_rhs(const double* mx, size_t mx_stride, const double* res,
                          size_t res_stride, int p, int nres, double c, double* rhs,
                          size_t rhs_stride, int B, hipStream_t st);

// b[s][ids[i]][t] = in[s][i][t] for B slices (float32, or bf16 bits when
// bf16): a delivered block's rows placed into a [B][n_angles][R] sinogram.
hipError_t launch_scatter_rows(const void* in, int bf16, int n_angles, int R, int B,
                               const AngleList& ids, void* b, hipStream_t st);

// Fixed forward scratch of the allocation-free projection: its capacity in
// floats, its set-up on the current device (hipGetSymbolAddress, once per
// device; slim_init calls it), and its device address on device dev (NULL
// before the set-up).  Concurrent users of one device share the array.
size_t forward_scratch_floats();
hipError_t forward_scratch_setup();
float* forward_scratch(int dev);

// Record msg as the library's last error message and return s.
slim_status set_error(slim_status s, const std::string& msg);


}  // namespace slim
