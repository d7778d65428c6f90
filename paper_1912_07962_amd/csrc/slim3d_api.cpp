// C ABI of the 3D parallel-beam slimLS path (include/slim3d.h): context,
// direction table, memory window and the host loop of the step's CG.
#include <cmath>
#include <deque>
#include <string>
#include <vector>

#include "../../include/slim3d.h"
#include "slim3d_internal.h"

using namespace slim;

namespace {

constexpr int kCtlWords = 4;     // done, iterations, breakdown, pad
constexpr int kNormGroup = 512;  // back-projector norm partials summed per group
constexpr int kChunk = 4;        // CG iterations enqueued between reads of the stop flag

#define HIP3_TRY(expr)                                                              \
  do {                                                                              \
    hipError_t _e = (expr);                                                         \
    if (_e != hipSuccess)                                                           \
      return set_error(SLIM_EDEVICE, std::string(#expr) + ": " + hipGetErrorString(_e)); \
  } while (0)

template <typename T>
hipError_t dalloc(T** p, size_t count) {
  *p = nullptr;
  if (count == 0) return hipSuccess;
  return hipMalloc((void**)p, count * sizeof(T));
}

}  // namespace

struct slim3d_ctx {
  int N = 0, n_dirs = 0, n = 0, r = 0, g = 1;
  double lam = 0.0;
  slim_opts o{};
  hipStream_t st = nullptr;
  int64_t nvox = 0, ell = 0, pmax = 0;

  std::vector<DirGeom> h_geom;
  DirGeom* d_geom = nullptr;

  const float* b = nullptr;
  float* x = nullptr;
  const float* x_true = nullptr;
  bool bound = false;

  int k = 0;
  std::deque<int> window;                 // ring slots, oldest first
  std::vector<std::vector<int>> slot_ids; // direction ids per slot

  double* d_e = nullptr;      // Gram right-hand side [pmax]: zeros, then the residual
  double* d_r = nullptr;      // CG residual          [pmax]
  double* d_pd = nullptr;     // CG direction         [pmax]
  double* d_q = nullptr;      // (M M^T + lam I) pd   [pmax]
  double* d_z = nullptr;      // solution             [pmax]
  // padded volume layouts of the three major axes (lay_floats(N) floats
  // each), read by the forward projector for directions of that major axis:
  // copies of x for the residual, M^T pd in the CG, copies of the caller's
  // volume in slim3d_project
  float* d_lay[3] = {nullptr, nullptr, nullptr};
  double* d_dots = nullptr;   // forward partial dots
  double* d_part = nullptr;   // forward per-segment ray sums, for up to wmax directions
  int wmax = 0;               // directions of the largest window, (r+1) g
  double* d_parts = nullptr;  // vector-kernel partial sums (two sets)
  int nparts = 0;
  bool jacobi = true;         // CG preconditioned by the Gram diagonal's inverse
  double* d_minv = nullptr;   // that inverse for the window's rays [pmax]
  double* d_sc = nullptr;     // CG scalars
  int* d_ctl = nullptr;       // CG stop flag, iterations, breakdown
  double* d_bparts = nullptr; // back-projector norm partials, padded to groups of 512
  double* d_btmp = nullptr;   // per-group norm sums
  int64_t nbgroups = 0;
  double* d_norms = nullptr;  // [3]
  int* h_ctl = nullptr;       // pinned [kCtlWords]
  double* h_out = nullptr;    // pinned: norms [3], rr, rr0
  Profiler prof;

  ~slim3d_ctx() {
    (void)hipFree(d_geom);
    (void)hipFree(d_e);
    (void)hipFree(d_r);
    (void)hipFree(d_pd);
    (void)hipFree(d_q);
    (void)hipFree(d_z);
    for (float* l : d_lay) (void)hipFree(l);
    (void)hipFree(d_dots);
    (void)hipFree(d_part);
    (void)hipFree(d_parts);
    (void)hipFree(d_minv);
    (void)hipFree(d_sc);
    (void)hipFree(d_ctl);
    (void)hipFree(d_bparts);
    (void)hipFree(d_btmp);
    (void)hipFree(d_norms);
    if (h_ctl) (void)hipHostFree(h_ctl);
    if (h_out) (void)hipHostFree(h_out);
    prof.release();
  }
};

namespace {

slim_status check_dir_ids(const slim3d_ctx* c, const int32_t* ids, int n, bool allow_repeat) {
  if (!ids || n <= 0) return set_error(SLIM_EINVAL, "direction id list is empty or NULL");
  if (n > kMaxList) return set_error(SLIM_EINVAL, "too many direction ids in one call");
  for (int i = 0; i < n; ++i) {
    if (ids[i] < 0 || ids[i] >= c->n_dirs)
      return set_error(SLIM_EINVAL, "direction id " + std::to_string(ids[i]) + " out of range");
    if (!allow_repeat)
      for (int j = 0; j < i; ++j)
        if (ids[j] == ids[i]) return set_error(SLIM_EINVAL, "duplicate direction id in a block");
  }
  return SLIM_OK;
}

// Bit m set when a direction of the list has major axis m.
int majors_of(const slim3d_ctx* c, const DirList& l) {
  int mask = 0;
  for (int i = 0; i < l.n; ++i) mask |= 1 << c->h_geom[l.id[i]].m;
  return mask;
}

// The padded copies of a standard-layout volume x that the forward
// projector reads for the majors in mask.
slim_status relayout_for(slim3d_ctx* c, const float* x, int mask) {
  for (int m = 0; m < 3; ++m)
    if (mask & (1 << m)) HIP3_TRY(launch_relayout3(x, c->d_lay[m], c->N, m, c->st));
  return SLIM_OK;
}

DirList make_dir_list(const int32_t* ids, int n) {
  DirList l;
  l.n = n;
  for (int i = 0; i < n; ++i) l.id[i] = ids[i];
  for (int i = n; i < kMaxList; ++i) l.id[i] = 0;
  return l;
}

// Geometry of direction w (unit length): detector basis, major axis and the
// linear maps of DirGeom.
DirGeom make_geom(const double* w, int N) {
  DirGeom G{};
  const double nz = std::hypot(w[0], w[1]);
  if (nz < 1e-12) {
    G.eu[0] = 1.0;
    G.eu[1] = 0.0;
    G.eu[2] = 0.0;
  } else {
    G.eu[0] = -w[1] / nz;
    G.eu[1] = w[0] / nz;
    G.eu[2] = 0.0;
  }
  // e_v = w x e_u
  G.ev[0] = w[1] * G.eu[2] - w[2] * G.eu[1];
  G.ev[1] = w[2] * G.eu[0] - w[0] * G.eu[2];
  G.ev[2] = w[0] * G.eu[1] - w[1] * G.eu[0];
  int m = 0;
  for (int i = 1; i < 3; ++i)
    if (std::fabs(w[i]) > std::fabs(w[m])) m = i;
  const int a = m == 0 ? 1 : 0;
  const int b = m == 2 ? 1 : 2;
  G.m = m;
  G.a = a;
  G.b = b;
  G.sa = w[a] / w[m];
  G.sb = w[b] / w[m];
  G.La[0] = G.eu[a] - G.eu[m] * G.sa;
  G.La[1] = G.ev[a] - G.ev[m] * G.sa;
  G.Lb[0] = G.eu[b] - G.eu[m] * G.sb;
  G.Lb[1] = G.ev[b] - G.ev[m] * G.sb;
  G.scale = (2.0 / N) / std::fabs(w[m]);
  G.wu = std::fabs(G.eu[a]) + std::fabs(G.eu[b]);
  G.wv = std::fabs(G.ev[a]) + std::fabs(G.ev[b]);
  return G;
}

// Sum the back-projector's per-workgroup norm partials (fixed order).
slim_status reduce_norms(slim3d_ctx* c) {
  HIP3_TRY(launch_reduce3(c->d_bparts, kNormGroup, (int)c->nbgroups, c->d_btmp, c->st));
  HIP3_TRY(launch_reduce3(c->d_btmp, (int)c->nbgroups, 1, c->d_norms, c->st));
  return SLIM_OK;
}

slim_status do_step3(slim3d_ctx* c, const int32_t* ids, slim_step_info* info) {
  const int S = c->r + 1;
  // the new window, committed to the context once the step's work is enqueued
  std::deque<int> win = c->window;
  const int slot = c->k % S;
  if ((int)win.size() == S) win.pop_front();
  win.push_back(slot);
  std::vector<std::vector<int>> slots = c->slot_ids;
  slots[slot].assign(ids, ids + c->g);
  DirList wl;
  wl.n = 0;
  for (int sl : win)
    for (int d : slots[sl]) wl.id[wl.n++] = d;
  for (int i = wl.n; i < kMaxList; ++i) wl.id[i] = 0;
  const int W = (int)win.size();
  const int64_t p = (int64_t)W * c->ell;

  // 1. residual of the new block into the last rows of the right-hand side
  if (c->prof.on) HIP3_TRY(c->prof.begin(K_RESID, c->st));
  {
    Fwd3Args fa;
    fa.geom = c->d_geom;
    fa.ids = make_dir_list(ids, c->g);
    fa.N = c->N;
    fa.n = c->n;
    slim_status s = relayout_for(c, c->x, majors_of(c, fa.ids));
    if (s != SLIM_OK) return s;
    for (int m = 0; m < 3; ++m) fa.lay[m] = c->d_lay[m];
    fa.sub = c->b;
    fa.out64 = c->d_e + (p - c->ell);
    fa.part = c->d_part;
    HIP3_TRY(launch_fwd3(fa, c->st));
  }
  if (p > c->ell) HIP3_TRY(hipMemsetAsync(c->d_e, 0, sizeof(double) * (p - c->ell), c->st));
  if (c->prof.on) HIP3_TRY(c->prof.end(c->st));

  // 2. CG on (M M^T + lam I) z = e
  const double tol = c->o.pcg_tol;
  if (c->prof.on) HIP3_TRY(c->prof.begin(K_VEC, c->st));
  if (c->jacobi) HIP3_TRY(launch_diag3(c->d_geom, wl, c->N, c->n, c->lam, c->d_minv, c->st));
  const double* minv = c->jacobi ? c->d_minv : nullptr;
  HIP3_TRY(launch_cg3_init(c->d_e, minv, c->d_r, c->d_pd, c->d_z, (int)p, c->d_parts, c->nparts,
                           c->d_sc, c->d_ctl, tol * tol, c->st));
  if (c->prof.on) HIP3_TRY(c->prof.end(c->st));
  Back3Args bu;
  bu.geom = c->d_geom;
  bu.ids = wl;
  bu.N = c->N;
  bu.n = c->n;
  bu.v64 = c->d_pd;
  {  // u = M^T pd written in the layouts of the window's majors
    const int mask = majors_of(c, wl);
    for (int m = 0; m < 3; ++m) bu.lay[m] = (mask & (1 << m)) ? c->d_lay[m] : nullptr;
  }
  bu.mode = 0;
  bu.ctl = c->d_ctl;
  Fwd3Args fq;
  fq.geom = c->d_geom;
  fq.ids = wl;
  fq.N = c->N;
  fq.n = c->n;
  for (int m = 0; m < 3; ++m) fq.lay[m] = c->d_lay[m];
  fq.out64 = c->d_q;
  fq.pd = c->d_pd;
  fq.lam = c->lam;
  fq.dots = c->d_dots;
  fq.ctl = c->d_ctl;
  fq.part = c->d_part;
  const int nd = fwd3_num_workgroups(c->n, wl.n);
  int enq = 0;
  bool done = false;
  while (!done) {
    const int chunk = std::min(kChunk, c->o.pcg_max_iter - enq);
    for (int it = 0; it < chunk; ++it) {
      if (c->prof.on) HIP3_TRY(c->prof.begin(K_BACK, c->st));
      HIP3_TRY(launch_back3(bu, c->st));
      if (c->prof.on) HIP3_TRY(c->prof.end(c->st));
      if (c->prof.on) HIP3_TRY(c->prof.begin(K_FORWARD, c->st));
      HIP3_TRY(launch_fwd3(fq, c->st));
      if (c->prof.on) HIP3_TRY(c->prof.end(c->st));
      if (c->prof.on) HIP3_TRY(c->prof.begin(K_VEC, c->st));
      HIP3_TRY(launch_cg3_alpha(c->d_dots, nd, c->d_sc, c->d_ctl, c->st));
      HIP3_TRY(launch_cg3_update(c->d_z, c->d_r, c->d_pd, c->d_q, minv, (int)p, c->d_parts,
                                 c->d_sc, c->d_ctl, c->st));
      HIP3_TRY(launch_cg3_beta(c->d_r, minv, c->d_pd, (int)p, c->d_parts, c->d_sc, c->d_ctl,
                               c->st));
      if (c->prof.on) HIP3_TRY(c->prof.end(c->st));
    }
    enq += chunk;
    HIP3_TRY(hipMemcpyAsync(c->h_ctl, c->d_ctl, sizeof(int) * kCtlWords, hipMemcpyDeviceToHost,
                            c->st));
    HIP3_TRY(hipStreamSynchronize(c->st));
    if (c->prof.on) HIP3_TRY(c->prof.harvest());
    done = c->h_ctl[kCtlDone] != 0 || enq >= c->o.pcg_max_iter;
  }

  // 3. x -= M^T z over the window, float64 norms
  if (c->prof.on) HIP3_TRY(c->prof.begin(K_UPDATE, c->st));
  {
    Back3Args ba;
    ba.geom = c->d_geom;
    ba.ids = wl;
    ba.N = c->N;
    ba.n = c->n;
    ba.v64 = c->d_z;
    ba.x = c->x;
    ba.x_true = c->x_true;
    ba.partials = c->d_bparts;
    ba.mode = 1;
    HIP3_TRY(launch_back3(ba, c->st));
    slim_status s = reduce_norms(c);
    if (s != SLIM_OK) return s;
  }
  if (c->prof.on) HIP3_TRY(c->prof.end(c->st));
  // the step is enqueued: commit the window
  c->window = win;
  c->slot_ids = slots;
  c->k += 1;
  HIP3_TRY(hipMemcpyAsync(c->h_out, c->d_norms, sizeof(double) * 3, hipMemcpyDeviceToHost, c->st));
  HIP3_TRY(hipMemcpyAsync(c->h_out + 3, c->d_sc, sizeof(double) * 2, hipMemcpyDeviceToHost, c->st));
  HIP3_TRY(hipStreamSynchronize(c->st));
  if (c->prof.on) HIP3_TRY(c->prof.harvest());
  const int iters = c->h_ctl[kCtlIters];
  const double rr = c->h_out[3 + SC3_RR], rr0 = c->h_out[3 + SC3_RR0];
  const double relres = rr0 > 0.0 ? std::sqrt(rr / rr0) : 0.0;
  if (info) {
    info->step_norm = std::sqrt(c->h_out[0]);
    info->x_norm = std::sqrt(c->h_out[1]);
    info->err_norm = c->x_true ? std::sqrt(c->h_out[2]) : -1.0;
    info->k = c->k;
    info->pcg_iters = iters;
    info->pcg_relres = relres;
  }
  for (int q = 0; q < 3; ++q)
    if (!std::isfinite(c->h_out[q])) return set_error(SLIM_ENUMERIC, "non-finite norm");
  if (c->h_ctl[2] != 0)
    return set_error(SLIM_ENUMERIC, "non-finite CG right-hand side or breakdown (non-positive curvature)");
  if (relres > tol) return set_error(SLIM_ENOTCONV, "CG reached its iteration cap");
  return SLIM_OK;
}

}  // namespace

extern "C" {

slim_status slim3d_init(slim3d_ctx** out, int N, int n_dirs, const double* dirs, int n_det, int r,
                        double lambda, const slim_opts* opts) {
  if (!out) return set_error(SLIM_EINVAL, "out is NULL");
  *out = nullptr;
  slim_opts o;
  slim_default_opts(&o);
  if (opts) o = *opts;
  if (N < 2 || N > 1024) return set_error(SLIM_EINVAL, "N must be in [2, 1024]");
  if (n_dirs < 1) return set_error(SLIM_EINVAL, "n_dirs must be >= 1");
  if (!dirs) return set_error(SLIM_EINVAL, "dirs is NULL");
  if (n_det < 1 || n_det > 4096) return set_error(SLIM_EINVAL, "n_det must be in [1, 4096]");
  if (r < 0) return set_error(SLIM_EINVAL, "memory level r must be >= 0");
  if (!(lambda > 0.0) || !std::isfinite(lambda))
    return set_error(SLIM_EINVAL, "lambda must be positive and finite");
  const int g = o.angles_per_block;
  if (g < 1 || n_dirs % g != 0) return set_error(SLIM_EINVAL, "angles_per_block must divide n_dirs");
  if ((int64_t)(r + 1) * g > kMaxList)
    return set_error(SLIM_EINVAL, "(r+1)*angles_per_block exceeds 256");
  if (o.precision != SLIM_PREC_FP32) return set_error(SLIM_EINVAL, "3D path needs FP32 precision");
  if (o.gram_mode == SLIM_GRAM_CHOL)
    return set_error(SLIM_EINVAL, "3D path solves the Gram system by CG only");
  if (o.gram_mode < SLIM_GRAM_AUTO || o.gram_mode > SLIM_GRAM_JACOBI)
    return set_error(SLIM_EINVAL, "unknown gram_mode");
  if (o.tikhonov != 0.0) return set_error(SLIM_EINVAL, "3D path has no Tikhonov term");
  if (o.pcg_max_iter < 1 || !(o.pcg_tol > 0.0)) return set_error(SLIM_EINVAL, "bad CG settings");
  for (int d = 0; d < n_dirs; ++d) {
    const double* w = dirs + 3 * d;
    if (!std::isfinite(w[0]) || !std::isfinite(w[1]) || !std::isfinite(w[2]))
      return set_error(SLIM_EINVAL, "non-finite direction");
    const double len = std::sqrt(w[0] * w[0] + w[1] * w[1] + w[2] * w[2]);
    if (std::fabs(len - 1.0) > 1e-6) return set_error(SLIM_EINVAL, "directions must have unit length");
  }
  const int64_t ell = (int64_t)g * n_det * n_det;
  const int64_t pmax = (int64_t)(r + 1) * ell;
  if (pmax > (int64_t)1 << 30) return set_error(SLIM_EINVAL, "window has more than 2^30 rows");

  slim3d_ctx* c = new slim3d_ctx();
  c->N = N;
  c->n_dirs = n_dirs;
  c->n = n_det;
  c->r = r;
  c->g = g;
  c->lam = lambda;
  c->o = o;
  c->st = (hipStream_t)o.stream;
  c->nvox = (int64_t)N * N * N;
  c->ell = ell;
  c->pmax = pmax;
  c->slot_ids.assign(r + 1, std::vector<int>());
  c->h_geom.resize(n_dirs);
  for (int d = 0; d < n_dirs; ++d) c->h_geom[d] = make_geom(dirs + 3 * d, N);

  auto oom = [&](hipError_t e) -> slim_status {
    delete c;
    if (e == hipErrorOutOfMemory || e == hipErrorMemoryAllocation)
      return set_error(SLIM_ENOMEM, "device workspace does not fit");
    return set_error(SLIM_EDEVICE, std::string("allocation: ") + hipGetErrorString(e));
  };
  hipError_t e;
  c->nparts = 2 * cg3_num_parts((int)pmax);
  c->jacobi = o.gram_mode != SLIM_GRAM_PCG;
  const int64_t nbw = back3_num_workgroups(N);
  c->nbgroups = (nbw + kNormGroup - 1) / kNormGroup;
  if ((e = dalloc(&c->d_geom, n_dirs)) != hipSuccess) return oom(e);
  if ((e = dalloc(&c->d_e, pmax)) != hipSuccess) return oom(e);
  if ((e = dalloc(&c->d_r, pmax)) != hipSuccess) return oom(e);
  if ((e = dalloc(&c->d_pd, pmax)) != hipSuccess) return oom(e);
  if ((e = dalloc(&c->d_q, pmax)) != hipSuccess) return oom(e);
  if ((e = dalloc(&c->d_z, pmax)) != hipSuccess) return oom(e);
  for (float*& l : c->d_lay)
    if ((e = dalloc(&l, lay_floats(N))) != hipSuccess) return oom(e);
  c->wmax = (r + 1) * g;
  if ((e = dalloc(&c->d_dots, (size_t)fwd3_num_workgroups(n_det, c->wmax))) != hipSuccess) return oom(e);
  if ((e = dalloc(&c->d_part, fwd3_part_doubles(n_det, c->wmax))) != hipSuccess) return oom(e);
  if ((e = dalloc(&c->d_parts, (size_t)c->nparts)) != hipSuccess) return oom(e);
  if (c->jacobi && (e = dalloc(&c->d_minv, pmax)) != hipSuccess) return oom(e);
  if ((e = dalloc(&c->d_sc, SC3_COUNT)) != hipSuccess) return oom(e);
  if ((e = dalloc(&c->d_ctl, kCtlWords)) != hipSuccess) return oom(e);
  if ((e = dalloc(&c->d_bparts, (size_t)c->nbgroups * kNormGroup * 3)) != hipSuccess) return oom(e);
  if ((e = dalloc(&c->d_btmp, (size_t)c->nbgroups * 3)) != hipSuccess) return oom(e);
  if ((e = dalloc(&c->d_norms, 3)) != hipSuccess) return oom(e);
  if ((e = hipHostMalloc((void**)&c->h_ctl, sizeof(int) * kCtlWords, hipHostMallocDefault)) != hipSuccess) return oom(e);
  if ((e = hipHostMalloc((void**)&c->h_out, sizeof(double) * 8, hipHostMallocDefault)) != hipSuccess) return oom(e);
  if ((e = hipMemcpyAsync(c->d_geom, c->h_geom.data(), sizeof(DirGeom) * n_dirs,
                          hipMemcpyHostToDevice, c->st)) != hipSuccess) return oom(e);
  // the layouts' pads and the padding of the last norm group are never
  // written by a kernel
  for (float* l : c->d_lay)
    if ((e = hipMemsetAsync(l, 0, sizeof(float) * lay_floats(N), c->st)) != hipSuccess) return oom(e);
  if ((e = hipMemsetAsync(c->d_bparts, 0, sizeof(double) * c->nbgroups * kNormGroup * 3, c->st)) != hipSuccess) return oom(e);
  if ((e = hipMemsetAsync(c->d_ctl, 0, sizeof(int) * kCtlWords, c->st)) != hipSuccess) return oom(e);
  if ((e = hipStreamSynchronize(c->st)) != hipSuccess) return oom(e);
  *out = c;
  return SLIM_OK;
}

slim_status slim3d_set_data(slim3d_ctx* c, const float* b, float* x, const float* x_true) {
  if (!c) return set_error(SLIM_EINVAL, "ctx is NULL");
  if (!b || !x) return set_error(SLIM_EINVAL, "b and x must be non-NULL");
  c->b = b;
  c->x = x;
  c->x_true = x_true;
  c->bound = true;
  c->k = 0;
  c->window.clear();
  for (auto& s : c->slot_ids) s.clear();
  return SLIM_OK;
}

slim_status slim3d_step(slim3d_ctx* c, const int32_t* ids, int n_ids, slim_step_info* info) {
  if (!c) return set_error(SLIM_EINVAL, "ctx is NULL");
  if (n_ids != c->g) return set_error(SLIM_EINVAL, "n_ids must equal angles_per_block");
  slim_status s = check_dir_ids(c, ids, n_ids, false);
  if (s != SLIM_OK) return s;
  if (!c->bound) return set_error(SLIM_ESTATE, "no data bound (slim3d_set_data)");
  s = do_step3(c, ids, info);
  if (s == SLIM_EDEVICE) c->bound = false;   // rebind before the next step
  return s;
}

slim_status slim3d_project(slim3d_ctx* c, const int32_t* ids, int n_ids, const float* x,
                           float* out) {
  if (!c) return set_error(SLIM_EINVAL, "ctx is NULL");
  slim_status s = check_dir_ids(c, ids, n_ids, true);
  if (s != SLIM_OK) return s;
  if (!x || !out) return set_error(SLIM_EINVAL, "x and out must be non-NULL");
  Fwd3Args fa;
  fa.geom = c->d_geom;
  fa.ids = make_dir_list(ids, n_ids);
  fa.N = c->N;
  fa.n = c->n;
  s = relayout_for(c, x, majors_of(c, fa.ids));
  if (s != SLIM_OK) return s;
  for (int m = 0; m < 3; ++m) fa.lay[m] = c->d_lay[m];
  fa.part = c->d_part;
  // the partial-sum workspace holds wmax directions: launch in chunks
  const size_t img = (size_t)c->n * c->n;
  for (int i0 = 0; i0 < n_ids; i0 += c->wmax) {
    const int cnt = std::min(c->wmax, n_ids - i0);
    fa.ids = make_dir_list(ids + i0, cnt);
    fa.out32 = out + i0 * img;
    HIP3_TRY(launch_fwd3(fa, c->st));
  }
  return SLIM_OK;
}

slim_status slim3d_backproject(slim3d_ctx* c, const int32_t* ids, int n_ids, const float* v,
                               float* out) {
  if (!c) return set_error(SLIM_EINVAL, "ctx is NULL");
  slim_status s = check_dir_ids(c, ids, n_ids, true);
  if (s != SLIM_OK) return s;
  if (!v || !out) return set_error(SLIM_EINVAL, "v and out must be non-NULL");
  Back3Args ba;
  ba.geom = c->d_geom;
  ba.ids = make_dir_list(ids, n_ids);
  ba.N = c->N;
  ba.n = c->n;
  ba.v32 = v;
  ba.out = out;
  ba.mode = 0;
  HIP3_TRY(launch_back3(ba, c->st));
  return SLIM_OK;
}

slim_status slim3d_profile(slim3d_ctx* c, int on) {
  if (!c) return set_error(SLIM_EINVAL, "ctx is NULL");
  HIP3_TRY(hipStreamSynchronize(c->st));
  HIP3_TRY(c->prof.harvest());
  if (on) {
    for (int k = 0; k < K_COUNT; ++k) {
      c->prof.total_ms[k] = 0.0;
      c->prof.launches[k] = 0;
    }
  }
  c->prof.on = on != 0;
  return SLIM_OK;
}

slim_status slim3d_kernel_stats(slim3d_ctx* c, int kind, double* total_ms, int64_t* launches) {
  if (!c || !total_ms || !launches) return set_error(SLIM_EINVAL, "NULL argument");
  if (kind < 0 || kind >= K_COUNT) return set_error(SLIM_EINVAL, "unknown kernel kind");
  HIP3_TRY(hipStreamSynchronize(c->st));
  HIP3_TRY(c->prof.harvest());
  *total_ms = c->prof.total_ms[kind];
  *launches = c->prof.launches[kind];
  return SLIM_OK;
}

void slim3d_destroy(slim3d_ctx* c) {
  if (!c) return;
  (void)hipStreamSynchronize(c->st);
  delete c;
}

}  // extern "C"
