// C ABI of the slimLS library: argument checks, context and workspace, the
// per-step schedule of kernels, the solve loop and its sampler.
//
// One step (paper eq. (ram), (B_k) with C_k = I, alpha = 1/lambda):
//   1. res = A_k x - b_k                      forward projector, fp64 sums
//   2. z = (M M^T + lambda I)^{-1} [0;..;res]  explicit Gram + FP64 Cholesky,
//                                             or PCG with matrix-free M, M^T
//   3. x <- x - M^T z                         back-projection fused with the
//                                             update and fp64 norm partials
// The memory window M_k = [A_{k-r}; ...; A_k] is a ring of r+1 block slots;
// Gram blocks between a slot and the older slots are computed when the slot
// is filled and reused while both stay in the window.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <deque>
#include <map>
#include <memory>
#include <mutex>
#include <string>
#include <tuple>
#include <vector>

#include "slim_internal.h"
#include "pcg.h"
#include "cnn_internal.h"

using namespace slim;

namespace {

thread_local std::string g_last_error;

slim_status fail(slim_status s, const std::string& msg) {
  g_last_error = msg;
  return s;
}

#define HIP_TRY(expr)                                                                   \
  do {                                                                                  \
    hipError_t _e = (expr);                                                             \
    if (_e != hipSuccess)                                                               \
      return fail(SLIM_EDEVICE, std::string(#expr) + ": " + hipGetErrorString(_e));     \
  } while (0)

template <typename T>
hipError_t dalloc(T** p, size_t count) {
  *p = nullptr;
  if (count == 0) return hipSuccess;
  return hipMalloc((void**)p, count * sizeof(T));
}

// SplitMix64 (Steele, Lea, Flood 2014), k-th output for a seed.
uint64_t splitmix64(uint64_t seed, uint64_t k) {
  uint64_t z = seed + k * 0x9E3779B97F4A7C15ull;
  z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
  z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
  return z ^ (z >> 31);
}

// Fisher-Yates shuffle of 0..M-1 for epoch e, driven by outputs
// e*(M-1)+1 ... of the seed; j = floor(u * (i+1) / 2^64).
std::vector<int> epoch_order(int M, int e, uint64_t seed) {
  std::vector<int> perm(M);
  for (int i = 0; i < M; ++i) perm[i] = i;
  uint64_t k = (uint64_t)e * (uint64_t)(M - 1);
  for (int i = M - 1; i >= 1; --i) {
    ++k;
    const uint64_t u = splitmix64(seed, k);
    const uint64_t j = (uint64_t)(((unsigned __int128)u * (unsigned __int128)(i + 1)) >> 64);
    std::swap(perm[i], perm[(int)j]);
  }
  return perm;
}

}  // namespace

slim_status slim::set_error(slim_status s, const std::string& msg) { return fail(s, msg); }

struct slim_ctx {
  int N = 0, B = 1, n_angles = 0, R = 0, r = 0, g = 1;
  double lam = 0.0;
  slim_opts o{};
  hipStream_t st = nullptr;
  int dev = 0;  // device current at slim_init
  int mode = SLIM_GRAM_CHOL;
  int64_t ell = 0, pmax = 0;

  std::vector<AngleGeom> h_geom;
  AngleGeom* d_geom = nullptr;

  const void* b = nullptr;
  float* x = nullptr;
  const float* x_true = nullptr;
  bool bound = false;

  // iteration state
  int k = 0;
  std::deque<int> window;                 // ring slots, oldest first
  std::vector<std::vector<int>> slot_ids; // angle ids per slot
  int epoch = 0, pos = 0;                 // solve sampler position

  // workspace
  double* d_res64 = nullptr;   // [B][ell]
  double* d_tiles = nullptr;   // [(r+1)^2][ell][ell]
  double* d_G = nullptr;       // [pmax][pmax]
  double* d_cholwork = nullptr;// inverse of a diagonal block (Cholesky scratch)
  double* d_ysolve = nullptr;  // [B][pmax] triangular-solve scratch
  double* d_z = nullptr;       // [B][pmax]
  double* d_mx = nullptr;      // [B][pmax] M x of the window (slimTik)
  double* d_rhs = nullptr;     // [B][pmax] Gram right-hand sides (slimTik)
  int* d_info = nullptr;
  double* d_partials = nullptr;
  double* d_norms = nullptr;   // [B][3]
  float* d_xT = nullptr;       // [B][N][N]
  float* d_tmp = nullptr;      // [B][N][N] scratch image (public projector)
  float* d_gather = nullptr;   // sinogram rows of an angle list [B][n][R]
  size_t gather_cap = 0;       // floats allocated in d_gather
  float* d_fpart = nullptr;    // forward projector partial sums
  size_t fpart_cap = 0;        // floats allocated in d_fpart
  uint16_t* d_xs = nullptr;    // bf16 shadow of x        [B][N][N] (precision BF16)
  uint16_t* d_xsT = nullptr;   // bf16 shadow of x^T      [B][N][N] (precision BF16)
  PcgWork pcg{};
  Profiler prof;
  ProjTune tune;               // projector launch shape (zeros: built-in rules)
  std::map<int, ProjTune> tune_by_n;  // tuned shapes per angle-list size

  const ProjTune& tune_for(int n) const {
    auto it = tune_by_n.find(n);
    return it != tune_by_n.end() ? it->second : tune;
  }

  // streaming data (slim_set_data with b == NULL): blocks arrive with
  // slim_step_data, are copied on copy_st into one of two staging buffers and
  // placed into d_bstream on the step's stream
  bool streaming = false;
  void* d_bstream = nullptr;              // [B][n_angles][R] sinogram
  void* d_stage[2] = {nullptr, nullptr};  // [B][g][R] delivered blocks
  hipStream_t copy_st = nullptr;
  hipEvent_t ev_copied[2] = {nullptr, nullptr};
  hipEvent_t ev_used[2] = {nullptr, nullptr};
  bool used_pending[2] = {false, false};
  int stage_next = 0;

  double* h_norms = nullptr;   // pinned [B][3]
  bool norms_valid = false;    // h_norms holds the last step read back
  int* h_info = nullptr;       // pinned

  int last_pcg_iters = 0;
  double last_pcg_relres = 0.0;
  int total_pcg_iters = 0;

  ~slim_ctx() {
    (void)hipFree(d_geom);
    (void)hipFree(d_res64);
    (void)hipFree(d_tiles);
    (void)hipFree(d_G);
    (void)hipFree(d_cholwork);
    (void)hipFree(d_ysolve);
    (void)hipFree(d_z);
    (void)hipFree(d_mx);
    (void)hipFree(d_rhs);
    (void)hipFree(d_info);
    (void)hipFree(d_partials);
    (void)hipFree(d_norms);
    (void)hipFree(d_xT);
    (void)hipFree(d_tmp);
    (void)hipFree(d_fpart);
    (void)hipFree(d_gather);
    (void)hipFree(d_xs);
    (void)hipFree(d_xsT);
    pcg_free(pcg);
    prof.release();
    if (h_norms) (void)hipHostFree(h_norms);
    if (h_info) (void)hipHostFree(h_info);
    if (copy_st) (void)hipStreamSynchronize(copy_st);
    (void)hipFree(d_bstream);
    (void)hipFree(d_stage[0]);
    (void)hipFree(d_stage[1]);
    for (int i = 0; i < 2; ++i) {
      if (ev_copied[i]) (void)hipEventDestroy(ev_copied[i]);
      if (ev_used[i]) (void)hipEventDestroy(ev_used[i]);
    }
    if (copy_st) (void)hipStreamDestroy(copy_st);
  }

  size_t img_elems() const { return (size_t)N * N; }
  bool bf16() const { return o.precision == SLIM_PREC_BF16; }
  bool graphs() const { return o.use_graph != 0 && st != nullptr; }
  size_t sino_elems() const { return (size_t)n_angles * R; }
};

namespace {

// Damping of the k-th step (1-based).  Constant lambda = 1/alpha, or with the
// ramp of sec. 4.2 (alpha_k = k alpha / (r+1) for the first r+1 steps)
// lambda_k = lambda (r+1) / k while k <= r.
double lam_at(const slim_ctx* c, int k) {
  if (c->o.damping_ramp && k >= 1 && k <= c->r) return c->lam * (double)(c->r + 1) / (double)k;
  return c->lam;
}

slim_status check_ids(const slim_ctx* c, const int32_t* ids, int n, bool allow_repeat) {
  if (!ids || n <= 0) return fail(SLIM_EINVAL, "angle id list is empty or NULL");
  if (n > kMaxList) return fail(SLIM_EINVAL, "too many angle ids in one call");
  for (int i = 0; i < n; ++i) {
    if (ids[i] < 0 || ids[i] >= c->n_angles)
      return fail(SLIM_EINVAL, "angle id " + std::to_string(ids[i]) + " out of range");
    if (!allow_repeat)
      for (int j = 0; j < i; ++j)
        if (ids[j] == ids[i]) return fail(SLIM_EINVAL, "duplicate angle id in a block");
  }
  return SLIM_OK;
}

AngleList make_list(const int32_t* ids, int n) {
  AngleList l;
  l.n = n;
  for (int i = 0; i < n; ++i) l.id[i] = ids[i];
  for (int i = n; i < kMaxList; ++i) l.id[i] = 0;
  return l;
}

// Refresh the copies of x that the forward projector reads: x^T (float32),
// or the bf16 shadows of x and x^T in the bf16-storage variant.
slim_status transpose_slices(slim_ctx* c) {
  if (c->bf16())
    HIP_TRY(launch_transpose(c->x, nullptr, c->N, c->B, c->img_elems(), c->d_xs, c->d_xsT, c->st));
  else
    HIP_TRY(launch_transpose(c->x, c->d_xT, c->N, c->B, c->img_elems(), nullptr, nullptr, c->st));
  return SLIM_OK;
}

// Grow the forward projector's partial-sum workspace for a launch over the
// list l (all slices); synchronises the stream only when it grows.
slim_status ensure_fpart(slim_ctx* c, const AngleList& l) {
  const size_t need = forward_partial_floats(c->h_geom.data(), c->N, c->R, l, c->B, c->tune_for(l.n));
  if (need <= c->fpart_cap) return SLIM_OK;
  HIP_TRY(hipStreamSynchronize(c->st));
  HIP_TRY(hipFree(c->d_fpart));
  c->d_fpart = nullptr;
  c->fpart_cap = 0;
  hipError_t e = hipMalloc((void**)&c->d_fpart, need * sizeof(float));
  if (e != hipSuccess) return fail(SLIM_ENOMEM, "forward workspace does not fit");
  c->fpart_cap = need;
  return SLIM_OK;
}

FwdArgs base_fwd(const slim_ctx* c, const AngleList* l) {
  FwdArgs a;
  a.tune = c->tune_for(l->n);
  a.geom = c->d_geom;
  a.h_geom = c->h_geom.data();
  a.N = c->N;
  a.R = c->R;
  a.B = c->B;
  a.ids = l;
  a.img_stride = c->img_elems();
  a.partial = c->d_fpart;
  return a;
}

// Gram mode: z = G^{-1} e for every slice, G shared by the slices, e the
// last nres entries rhs (stride rhs_stride) after zeros.
slim_status gram_solve_chol(slim_ctx* c, int new_slot, double lam, const double* rhs,
                            size_t rhs_stride, int nres) {
  const int64_t ell = c->ell;
  const int W = (int)c->window.size();
  const int64_t p = (int64_t)W * ell;
  const int S = c->r + 1;
  // new slot's row of tiles
  if (c->prof.on) HIP_TRY(c->prof.begin(K_GRAM, c->st));
  AngleList na = make_list(c->slot_ids[new_slot].data(), c->g);
  for (int q : c->window) {
    AngleList nb = make_list(c->slot_ids[q].data(), c->g);
    double* T = c->d_tiles + ((int64_t)new_slot * S + q) * ell * ell;
    HIP_TRY(launch_gram(c->d_geom, c->N, c->R, na, nb, T, ell, c->st));
  }
  // assemble the lower triangle of G in window order (oldest first); the
  // window is consecutive ring slots, so one launch places every tile
  bool ring = true;
  for (int P = 0; P < W; ++P) ring = ring && c->window[P] == (c->window[0] + P) % S;
  if (ring && (int64_t)W * (W + 1) / 2 <= 65535 && ell <= 65535) {
    HIP_TRY(launch_tile_assemble(c->d_tiles, S, c->window[0], W, (int)ell, c->d_G, p, lam,
                                 c->st));
  } else {
    for (int P = 0; P < W; ++P)
      for (int Q = 0; Q <= P; ++Q) {
        const int sp = c->window[P], sq = c->window[Q];
        const double* T = c->d_tiles + ((int64_t)sp * S + sq) * ell * ell;
        HIP_TRY(launch_tile_copy(T, ell, c->d_G, p, (int)(P * ell), (int)(Q * ell), (int)ell,
                                 (int)ell, lam, P == Q, c->st));
      }
  }
  if (c->prof.on) HIP_TRY(c->prof.end(c->st));
  if (c->prof.on) HIP_TRY(c->prof.begin(K_CHOL, c->st));
  HIP_TRY(hipMemsetAsync(c->d_info, 0, sizeof(int), c->st));
  HIP_TRY(launch_cholesky(c->d_G, p, (int)p, c->d_info, c->d_cholwork, c->st));
  HIP_TRY(launch_chol_solve(c->d_G, p, (int)p, nres, c->d_cholwork, rhs, rhs_stride, c->d_z, c->pmax,
                            c->d_ysolve, c->B, c->st));
  if (c->prof.on) HIP_TRY(c->prof.end(c->st));
  return SLIM_OK;
}

// One step in two halves around the Gram solve, so that a group of contexts
// can interleave their CG solves.  A StepState must not move between
// step_begin and step_end (its CG run points into itself).
struct StepState {
  AngleList blk, win;
  int slot = 0;
  double lam = 0.0;  // diagonal shift of this step's Gram system
  float shrink = 0.f;  // slimTik: c of s = M^T z + c x
  bool pcg = false;
  PcgRun run;
};

// The window after a step with block ids (slot k mod (r+1); the oldest
// block leaves once r+1 are held), and the angle lists of the new block and
// of that window, without changing the context.
void plan_window(const slim_ctx* c, const int32_t* ids, StepState& ss, std::deque<int>& win) {
  const int S = c->r + 1;
  ss.slot = c->k % S;
  win = c->window;
  if ((int)win.size() == S) win.pop_front();
  win.push_back(ss.slot);
  ss.blk = make_list(ids, c->g);
  ss.win.n = 0;
  for (int sl : win) {
    if (sl == ss.slot)
      for (int a = 0; a < c->g; ++a) ss.win.id[ss.win.n++] = ids[a];
    else
      for (int a : c->slot_ids[sl]) ss.win.id[ss.win.n++] = a;
  }
  for (int i = ss.win.n; i < kMaxList; ++i) ss.win.id[i] = 0;
}

// Host work of a step that can fail without touching the iteration state:
// the forward projector's workspace for the new block and the window.
slim_status step_prepare(slim_ctx* c, const StepState& ss) {
  slim_status s = ensure_fpart(c, ss.blk);
  if (s == SLIM_OK && (c->mode == SLIM_GRAM_PCG || c->o.tikhonov > 0.0)) s = ensure_fpart(c, ss.win);
  return s;
}

// Everything up to the Gram solve.  The window is committed only after
// step_prepare succeeded, so a refused step (workspace that does not fit)
// leaves the context as it was; a failing device call (SLIM_EDEVICE) leaves
// the context unbound (the caller rebinds with slim_set_data).
slim_status step_begin(slim_ctx* c, const int32_t* ids, StepState& ss) {
  std::deque<int> win;
  plan_window(c, ids, ss, win);
  ss.lam = lam_at(c, c->k + 1);
  const int64_t ell = c->ell;
  {
    slim_status s = step_prepare(c, ss);
    if (s != SLIM_OK) return s;
  }
  c->window = win;
  c->slot_ids[ss.slot].assign(ids, ids + c->g);
  if (c->prof.on && c->prof.used > 4096) {
    HIP_TRY(hipStreamSynchronize(c->st));
    HIP_TRY(c->prof.harvest());
  }
  // 1. residual of the new block, all slices in one launch
  if (c->prof.on) HIP_TRY(c->prof.begin(K_RESID, c->st));
  {
    FwdArgs fa = base_fwd(c, &ss.blk);
    fa.img = c->bf16() ? (const void*)c->d_xs : (const void*)c->x;
    fa.imgT = c->bf16() ? (const void*)c->d_xsT : (const void*)c->d_xT;
    fa.img_bf16 = c->bf16();
    fa.sub = c->b;
    fa.sub_stride = c->sino_elems();
    fa.sub_bf16 = c->bf16();
    fa.out64 = c->d_res64;
    fa.out_stride = ell;
    HIP_TRY(launch_forward(fa, c->st));
  }
  if (c->prof.on) HIP_TRY(c->prof.end(c->st));
  // slimTik (eq. (slimTik), L = I): shift mu = lambda_k + W tau with
  // tau = tik^2 / M, right-hand side [0; res] - (tau / mu) M x
  const double* rhs = c->d_res64;
  size_t rhs_stride = ell;
  int nres = (int)ell;
  if (c->o.tikhonov > 0.0) {
    const int W = (int)c->window.size();
    const int p = (int)(W * ell);
    const double tau = c->o.tikhonov * c->o.tikhonov / (double)(c->n_angles / c->g);
    const double mu = ss.lam + W * tau;
    const double cs = tau / mu;
    ss.lam = mu;
    ss.shrink = (float)cs;
    FwdArgs fa = base_fwd(c, &ss.win);
    fa.img = c->x;
    fa.imgT = c->d_xT;
    fa.out64 = c->d_mx;
    fa.out_stride = c->pmax;
    if (c->prof.on) HIP_TRY(c->prof.begin(K_RESID, c->st));
    HIP_TRY(launch_forward(fa, c->st));
    HIP_TRY(launch_tik_rhs(c->d_mx, c->pmax, c->d_res64, ell, p, (int)ell, cs, c->d_rhs, c->pmax,
                           c->B, c->st));
    if (c->prof.on) HIP_TRY(c->prof.end(c->st));
    rhs = c->d_rhs;
    rhs_stride = c->pmax;
    nres = p;
  }
  // 2. Gram system: solved here (Cholesky) or started (CG)
  ss.pcg = c->mode == SLIM_GRAM_PCG;
  if (!ss.pcg) return gram_solve_chol(c, ss.slot, ss.lam, rhs, rhs_stride, nres);
  hipError_t e = pcg_begin(ss.run, c->pcg, c->d_geom, c->h_geom.data(), c->d_fpart, c->N, c->R,
                           c->B, ss.win, c->tune_for(ss.win.n), ss.lam, rhs, rhs_stride, nres, c->d_z,
                           c->pmax, c->o.pcg_tol, c->o.pcg_max_iter, &c->prof, c->st);
  if (e != hipSuccess) return fail(SLIM_EDEVICE, std::string("pcg: ") + hipGetErrorString(e));
  return SLIM_OK;
}

slim_status step_end(slim_ctx* c, StepState& ss, slim_step_info* info) {
  int pcg_it = 0;
  double pcg_rel = 0.0;
  if (ss.pcg) {  // the CG's final state travels with the step's other results
    hipError_t e = pcg_finish_async(ss.run);
    if (e != hipSuccess) return fail(SLIM_EDEVICE, std::string("pcg: ") + hipGetErrorString(e));
  }
  // 3. update every slice
  const int nwg = back_num_workgroups(c->N);
  if (c->prof.on) HIP_TRY(c->prof.begin(K_UPDATE, c->st));
  {
    BackArgs ba;
    ba.tune = c->tune_for(ss.win.n);
    ba.geom = c->d_geom;
    ba.N = c->N;
    ba.R = c->R;
    ba.B = c->B;
    ba.ids = &ss.win;
    ba.v64 = c->d_z;
    ba.v_stride = c->pmax;
    ba.x = c->x;
    ba.xT = c->bf16() ? nullptr : c->d_xT;
    ba.x_true = c->x_true;
    ba.img_stride = c->img_elems();
    ba.partials = c->d_partials;
    ba.mode = 1;
    ba.xs = c->bf16() ? c->d_xs : nullptr;
    ba.xsT = c->bf16() ? c->d_xsT : nullptr;
    ba.shrink = ss.shrink;
    HIP_TRY(launch_back(ba, c->st));
    HIP_TRY(launch_reduce3(c->d_partials, nwg, c->B, c->d_norms, c->st));
  }
  if (c->prof.on) HIP_TRY(c->prof.end(c->st));
  c->k += 1;
  if (info) {
    HIP_TRY(hipMemcpyAsync(c->h_norms, c->d_norms, sizeof(double) * 3 * c->B,
                           hipMemcpyDeviceToHost, c->st));
    HIP_TRY(hipMemcpyAsync(c->h_info, c->d_info, sizeof(int), hipMemcpyDeviceToHost, c->st));
  }
  if (info || ss.pcg) {
    HIP_TRY(hipStreamSynchronize(c->st));
    if (c->prof.on) HIP_TRY(c->prof.harvest());
  }
  if (ss.pcg) pcg_report(ss.run, &pcg_it, &pcg_rel);
  c->last_pcg_iters = pcg_it;
  c->last_pcg_relres = pcg_rel;
  c->total_pcg_iters += pcg_it;
  if (!info) return SLIM_OK;
  c->norms_valid = true;
  int best = 0;
  for (int sl = 1; sl < c->B; ++sl)
    if (c->h_norms[3 * sl] > c->h_norms[3 * best]) best = sl;
  info->step_norm = std::sqrt(c->h_norms[3 * best + 0]);
  info->x_norm = std::sqrt(c->h_norms[3 * best + 1]);
  info->err_norm = c->x_true ? std::sqrt(c->h_norms[3 * best + 2]) : -1.0;
  info->k = c->k;
  info->pcg_iters = pcg_it;
  info->pcg_relres = pcg_rel;
  for (int sl = 0; sl < c->B; ++sl)
    for (int q = 0; q < 3; ++q)
      if (!std::isfinite(c->h_norms[3 * sl + q])) return fail(SLIM_ENUMERIC, "non-finite norm");
  if (c->mode == SLIM_GRAM_CHOL && *c->h_info != 0)
    return fail(SLIM_ENUMERIC, "Cholesky pivot " + std::to_string(*c->h_info - 1) + " not positive");
  if (c->mode == SLIM_GRAM_PCG && !std::isfinite(pcg_rel))
    return fail(SLIM_ENUMERIC, "non-finite CG right-hand side (data or iterate not finite)");
  if (c->mode == SLIM_GRAM_PCG && pcg_rel > c->o.pcg_tol)
    return fail(SLIM_ENOTCONV, "CG reached its iteration cap");
  return SLIM_OK;
}

slim_status do_step_inner(slim_ctx* c, const int32_t* ids, slim_step_info* info) {
  StepState ss;
  slim_status s = step_begin(c, ids, ss);
  if (s != SLIM_OK) return s;
  while (ss.pcg && !ss.run.done) {
    hipError_t e = pcg_enqueue(ss.run, c->graphs());
    if (e == hipSuccess) e = pcg_poll(ss.run);
    if (e != hipSuccess) return fail(SLIM_EDEVICE, std::string("pcg: ") + hipGetErrorString(e));
  }
  return step_end(c, ss, info);
}

// A device failure inside a step leaves the window and the device state out
// of step with each other: the context must be rebound before the next step.
slim_status do_step(slim_ctx* c, const int32_t* ids, slim_step_info* info) {
  const slim_status s = do_step_inner(c, ids, info);
  if (s == SLIM_EDEVICE) c->bound = false;
  return s;
}

}  // namespace

extern "C" {

const char* slim_strerror(slim_status s) {
  // a C caller may pass any int: read the representation, not an enum value
  // that C++ need not be able to hold
  int v = 0;
  std::memcpy(&v, &s, sizeof v);
  switch (v) {
    case SLIM_OK: return "ok";
    case SLIM_EINVAL: return "invalid argument";
    case SLIM_ENOMEM: return "out of device memory";
    case SLIM_EDEVICE: return "device error";
    case SLIM_ENUMERIC: return "numerical failure";
    case SLIM_ENOTCONV: return "iteration did not converge";
    case SLIM_ESTATE: return "invalid state";
  }
  return "unknown status";
}

const char* slim_last_error(void) { return g_last_error.c_str(); }

slim_status slim_default_opts(slim_opts* o) {
  if (!o) return fail(SLIM_EINVAL, "opts is NULL");
  o->angles_per_block = 1;
  o->precision = SLIM_PREC_FP32;
  o->gram_mode = SLIM_GRAM_AUTO;
  o->chol_max_p = 8192;
  o->pcg_max_iter = 1000;
  o->pcg_tol = 1e-6;
  o->check_every = 1;
  o->seed = 0;
  o->stream = nullptr;
  o->use_graph = 1;
  o->damping_ramp = 0;
  o->tikhonov = 0.0;
  return SLIM_OK;
}

slim_status slim_init(slim_ctx** out, const slim_grid* grid, int n_angles, const double* angles,
                      int n_rays, int r, double lambda, const slim_opts* opts) {
  g_last_error.clear();
  if (!out) return fail(SLIM_EINVAL, "out is NULL");
  *out = nullptr;
  if (!grid) return fail(SLIM_EINVAL, "grid is NULL");
  slim_opts o;
  slim_default_opts(&o);
  if (opts) o = *opts;
  if (grid->N < 2 || grid->N > 8192) return fail(SLIM_EINVAL, "N must be in [2, 8192]");
  if (grid->n_slices < 1) return fail(SLIM_EINVAL, "n_slices must be >= 1");
  if (n_angles < 1) return fail(SLIM_EINVAL, "n_angles must be >= 1");
  if (n_rays < 1 || n_rays > 4096) return fail(SLIM_EINVAL, "n_rays must be in [1, 4096]");
  if (r < 0) return fail(SLIM_EINVAL, "memory level r must be >= 0");
  if (!(lambda > 0.0) || !std::isfinite(lambda)) return fail(SLIM_EINVAL, "lambda must be positive and finite");
  const int g = o.angles_per_block;
  if (g < 1 || n_angles % g != 0) return fail(SLIM_EINVAL, "angles_per_block must divide n_angles");
  if ((int64_t)(r + 1) * g > kMaxList) return fail(SLIM_EINVAL, "(r+1)*angles_per_block exceeds 256");
  if (o.precision != SLIM_PREC_FP32 && o.precision != SLIM_PREC_BF16)
    return fail(SLIM_EINVAL, "unknown precision");
  if (o.gram_mode == SLIM_GRAM_JACOBI) return fail(SLIM_EINVAL, "Jacobi preconditioning is a 3D option");
  if (o.gram_mode < SLIM_GRAM_AUTO || o.gram_mode > SLIM_GRAM_PCG) return fail(SLIM_EINVAL, "unknown gram_mode");
  if (o.check_every < 1) return fail(SLIM_EINVAL, "check_every must be >= 1");
  if (o.damping_ramp != 0 && o.damping_ramp != 1) return fail(SLIM_EINVAL, "damping_ramp must be 0 or 1");
  if (!(o.tikhonov >= 0.0) || !std::isfinite(o.tikhonov)) return fail(SLIM_EINVAL, "tikhonov must be >= 0 and finite");
  if (o.tikhonov > 0.0 && o.precision != SLIM_PREC_FP32) return fail(SLIM_EINVAL, "tikhonov needs FP32 precision");
  if (o.pcg_max_iter < 1 || !(o.pcg_tol > 0.0)) return fail(SLIM_EINVAL, "bad CG settings");
  if (angles) {
    for (int a = 0; a < n_angles; ++a)
      if (!std::isfinite(angles[a])) return fail(SLIM_EINVAL, "non-finite angle");
  }
  const int64_t ell = (int64_t)g * n_rays;
  const int64_t pmax = (int64_t)(r + 1) * ell;
  int mode = o.gram_mode;
  if (mode == SLIM_GRAM_AUTO) mode = (pmax <= o.chol_max_p && pmax <= 8192) ? SLIM_GRAM_CHOL : SLIM_GRAM_PCG;
  if (mode == SLIM_GRAM_CHOL && pmax > 8192)
    return fail(SLIM_EINVAL, "explicit Gram needs (r+1)*g*n_rays <= 8192; use PCG");

  slim_ctx* c = new slim_ctx();
  c->N = grid->N;
  c->B = grid->n_slices;
  c->n_angles = n_angles;
  c->R = n_rays;
  c->r = r;
  c->g = g;
  c->lam = lambda;
  c->o = o;
  c->st = (hipStream_t)o.stream;
  c->mode = mode;
  c->ell = ell;
  c->pmax = pmax;
  c->slot_ids.assign(r + 1, std::vector<int>());

  c->h_geom.resize(n_angles);
  for (int a = 0; a < n_angles; ++a) {
    const double th = angles ? angles[a] : (double)a * (M_PI / (double)n_angles);
    const double cs = std::cos(th), sn = std::sin(th);
    const double d = std::max(std::fabs(cs), std::fabs(sn));
    AngleGeom& G = c->h_geom[a];
    G.c = cs;
    G.s = sn;
    G.hd = (float)((2.0 / c->N) / d);
    G.invd = (float)(1.0 / d);
    G.colmajor = std::fabs(sn) > std::fabs(cs) ? 1 : 0;
    G.pad = 0;
    fwd_angle_consts(G, c->N, c->R);
  }
  auto oom = [&](hipError_t e) -> slim_status {
    delete c;
    if (e == hipErrorOutOfMemory || e == hipErrorMemoryAllocation)
      return fail(SLIM_ENOMEM, "device workspace does not fit");
    return fail(SLIM_EDEVICE, std::string("allocation: ") + hipGetErrorString(e));
  };
  hipError_t e;
  if ((e = hipGetDevice(&c->dev)) != hipSuccess) return oom(e);
  // the allocation-free projection's scratch: its address on this device
  if ((e = forward_scratch_setup()) != hipSuccess) return oom(e);
  const size_t nimg = c->img_elems() * c->B;
  if ((e = dalloc(&c->d_geom, n_angles)) != hipSuccess) return oom(e);
  if ((e = dalloc(&c->d_res64, (size_t)c->B * ell)) != hipSuccess) return oom(e);
  if ((e = dalloc(&c->d_z, (size_t)c->B * pmax)) != hipSuccess) return oom(e);
  if (o.tikhonov > 0.0) {
    if ((e = dalloc(&c->d_mx, (size_t)c->B * pmax)) != hipSuccess) return oom(e);
    if ((e = dalloc(&c->d_rhs, (size_t)c->B * pmax)) != hipSuccess) return oom(e);
  }
  if ((e = dalloc(&c->d_info, 1)) != hipSuccess) return oom(e);
  if ((e = dalloc(&c->d_partials, 3 * (size_t)c->B * back_num_workgroups(c->N))) != hipSuccess) return oom(e);
  if ((e = dalloc(&c->d_norms, 3 * (size_t)c->B)) != hipSuccess) return oom(e);
  if (o.precision == SLIM_PREC_BF16) {
    if ((e = dalloc(&c->d_xs, nimg)) != hipSuccess) return oom(e);
    if ((e = dalloc(&c->d_xsT, nimg)) != hipSuccess) return oom(e);
  } else {
    if ((e = dalloc(&c->d_xT, nimg)) != hipSuccess) return oom(e);
  }
  if ((e = dalloc(&c->d_tmp, nimg)) != hipSuccess) return oom(e);
  if (mode == SLIM_GRAM_CHOL) {
    if ((e = dalloc(&c->d_tiles, (size_t)(r + 1) * (r + 1) * ell * ell)) != hipSuccess) return oom(e);
    if ((e = dalloc(&c->d_G, (size_t)pmax * pmax)) != hipSuccess) return oom(e);
    if ((e = dalloc(&c->d_cholwork, chol_work_doubles(pmax))) != hipSuccess) return oom(e);
    if ((e = dalloc(&c->d_ysolve, (size_t)c->B * pmax)) != hipSuccess) return oom(e);
  } else {
    if ((e = pcg_alloc(c->pcg, c->N, c->B, pmax)) != hipSuccess) return oom(e);
  }
  if ((e = hipHostMalloc((void**)&c->h_norms, sizeof(double) * 3 * c->B, hipHostMallocDefault)) != hipSuccess) return oom(e);
  if ((e = hipHostMalloc((void**)&c->h_info, sizeof(int), hipHostMallocDefault)) != hipSuccess) return oom(e);
  if ((e = hipMemcpyAsync(c->d_geom, c->h_geom.data(), sizeof(AngleGeom) * n_angles,
                          hipMemcpyHostToDevice, c->st)) != hipSuccess) return oom(e);
  if ((e = hipMemsetAsync(c->d_info, 0, sizeof(int), c->st)) != hipSuccess) return oom(e);
  if ((e = hipStreamSynchronize(c->st)) != hipSuccess) return oom(e);
  *out = c;
  return SLIM_OK;
}

// Buffers, stream and events of streaming mode, created on first use.
// Device (or managed) memory: its producer may still be running on the
// context's stream, so such a block is read in that stream's order.
static bool on_device(const void* p) {
  hipPointerAttribute_t a;
  if (hipPointerGetAttributes(&a, p) != hipSuccess) {
    (void)hipGetLastError();  // unregistered host memory: clear the query's error
    return false;
  }
  return a.type == hipMemoryTypeDevice || a.type == hipMemoryTypeManaged;
}

static slim_status ensure_streaming(slim_ctx* c) {
  if (c->d_bstream) return SLIM_OK;
  const size_t esz = c->bf16() ? 2 : 4;
  hipError_t e;
  if ((e = hipMalloc(&c->d_bstream, esz * c->B * c->n_angles * c->R)) != hipSuccess ||
      (e = hipMalloc(&c->d_stage[0], esz * c->B * c->g * c->R)) != hipSuccess ||
      (e = hipMalloc(&c->d_stage[1], esz * c->B * c->g * c->R)) != hipSuccess) {
    (void)hipFree(c->d_bstream);
    (void)hipFree(c->d_stage[0]);
    (void)hipFree(c->d_stage[1]);
    c->d_bstream = c->d_stage[0] = c->d_stage[1] = nullptr;
    return fail(e == hipErrorOutOfMemory ? SLIM_ENOMEM : SLIM_EDEVICE,
                std::string("streaming buffers: ") + hipGetErrorString(e));
  }
  HIP_TRY(hipStreamCreateWithFlags(&c->copy_st, hipStreamNonBlocking));
  for (int i = 0; i < 2; ++i) {
    HIP_TRY(hipEventCreateWithFlags(&c->ev_copied[i], hipEventDisableTiming));
    HIP_TRY(hipEventCreateWithFlags(&c->ev_used[i], hipEventDisableTiming));
  }
  return SLIM_OK;
}

slim_status slim_set_data(slim_ctx* c, const void* b, void* x, const float* x_true) {
  if (!c) return fail(SLIM_EINVAL, "ctx is NULL");
  if (!x) return fail(SLIM_EINVAL, "x must be non-NULL");
  c->streaming = b == nullptr;
  if (c->streaming) {
    slim_status s = ensure_streaming(c);
    if (s != SLIM_OK) return s;
    const size_t esz = c->bf16() ? 2 : 4;
    HIP_TRY(hipMemsetAsync(c->d_bstream, 0, esz * c->B * c->n_angles * c->R, c->st));
    b = c->d_bstream;
  }
  c->b = b;
  c->x = (float*)x;
  c->x_true = x_true;
  c->bound = true;
  c->k = 0;
  c->norms_valid = false;
  c->window.clear();
  c->epoch = 0;
  c->pos = 0;
  c->total_pcg_iters = 0;
  return transpose_slices(c);
}

slim_status slim_set_lambda(slim_ctx* c, double lambda) {
  if (!c) return fail(SLIM_EINVAL, "ctx is NULL");
  if (!(lambda > 0.0) || !std::isfinite(lambda)) return fail(SLIM_EINVAL, "lambda must be positive and finite");
  c->lam = lambda;
  return SLIM_OK;
}

slim_status slim_step(slim_ctx* c, const int32_t* ids, int n_ids, slim_step_info* info) {
  if (!c) return fail(SLIM_EINVAL, "ctx is NULL");
  if (n_ids != c->g) return fail(SLIM_EINVAL, "n_ids must equal angles_per_block");
  slim_status s = check_ids(c, ids, n_ids, false);
  if (s != SLIM_OK) return s;
  if (!c->bound) return fail(SLIM_ESTATE, "no data bound (slim_set_data)");
  if (c->streaming) return fail(SLIM_ESTATE, "streaming context: pass each block's data to slim_step_data");
  return do_step(c, ids, info);
}

slim_status slim_step_data(slim_ctx* c, const int32_t* ids, int n_ids, const void* b_block,
                           slim_step_info* info) {
  if (!c) return fail(SLIM_EINVAL, "ctx is NULL");
  if (n_ids != c->g) return fail(SLIM_EINVAL, "n_ids must equal angles_per_block");
  if (!b_block) return fail(SLIM_EINVAL, "b_block is NULL");
  slim_status s = check_ids(c, ids, n_ids, false);
  if (s != SLIM_OK) return s;
  if (!c->bound || !c->streaming)
    return fail(SLIM_ESTATE, "no streaming data bound (slim_set_data with b = NULL)");
  const AngleList l = make_list(ids, c->g);
  if (on_device(b_block)) {  // placed directly, in the context stream's order
    HIP_TRY(launch_scatter_rows(b_block, c->bf16() ? 1 : 0, c->n_angles, c->R, c->B, l,
                                c->d_bstream, c->st));
    return do_step(c, ids, info);
  }
  const int k = c->stage_next;
  c->stage_next ^= 1;
  const size_t bytes = (size_t)(c->bf16() ? 2 : 4) * c->B * c->g * c->R;
  // the staging buffer is free once the step that used it two calls ago
  // has placed its rows
  if (c->used_pending[k]) HIP_TRY(hipStreamWaitEvent(c->copy_st, c->ev_used[k], 0));
  HIP_TRY(hipMemcpyAsync(c->d_stage[k], b_block, bytes, hipMemcpyHostToDevice, c->copy_st));
  HIP_TRY(hipEventRecord(c->ev_copied[k], c->copy_st));
  HIP_TRY(hipStreamWaitEvent(c->st, c->ev_copied[k], 0));
  HIP_TRY(launch_scatter_rows(c->d_stage[k], c->bf16() ? 1 : 0, c->n_angles, c->R, c->B, l,
                              c->d_bstream, c->st));
  HIP_TRY(hipEventRecord(c->ev_used[k], c->st));
  c->used_pending[k] = true;
  return do_step(c, ids, info);
}

slim_status slim_solve(slim_ctx* c, const void* b, void* x, const float* x_true, double tol,
                       int max_epochs, slim_solve_info* info) {
  if (!c) return fail(SLIM_EINVAL, "ctx is NULL");
  if (max_epochs < 1) return fail(SLIM_EINVAL, "max_epochs must be >= 1");
  if (!std::isfinite(tol)) return fail(SLIM_EINVAL, "tol must be finite");
  if (!b) return fail(SLIM_EINVAL, "b must be non-NULL");
  slim_status s = slim_set_data(c, b, x, x_true);
  if (s != SLIM_OK) return s;
  const int M = c->n_angles / c->g;
  slim_solve_info si{};
  si.err_last = -1.0;
  std::vector<int32_t> ids(c->g);
  bool done = false;
  for (int e = 0; e < max_epochs && !done; ++e) {
    si.epochs = e + 1;
    const std::vector<int> order = epoch_order(M, e, c->o.seed);
    for (int q = 0; q < M && !done; ++q) {
      for (int a = 0; a < c->g; ++a) ids[a] = order[q] * c->g + a;
      c->epoch = e;
      c->pos = q + 1;
      const bool check = ((c->k + 1) % c->o.check_every == 0) || (e == max_epochs - 1 && q == M - 1);
      slim_step_info st{};
      s = do_step(c, ids.data(), check ? &st : nullptr);
      if (s != SLIM_OK && s != SLIM_ENOTCONV) return s;
      si.steps = c->k;
      if (check) {
        si.rho_last = st.x_norm > 0 ? st.step_norm / st.x_norm : INFINITY;
        if (tol > 0 && c->k >= c->r + 1 && st.step_norm <= tol * st.x_norm) {
          si.converged = 1;
          done = true;
        }
      }
    }
  }
  si.pcg_iters = c->total_pcg_iters;
  if (info) *info = si;
  return SLIM_OK;
}

slim_status slim_project(slim_ctx* c, const int32_t* ids, int n_ids, const float* x, float* out) {
  if (!c) return fail(SLIM_EINVAL, "ctx is NULL");
  slim_status s = check_ids(c, ids, n_ids, true);
  if (s != SLIM_OK) return s;
  if (!x || !out) return fail(SLIM_EINVAL, "x and out must be non-NULL");
  const AngleList l = make_list(ids, n_ids);
  s = ensure_fpart(c, l);
  if (s != SLIM_OK) return s;
  // column-stepping angles stage bands of columns of x (no transposed copy)
  FwdArgs fa = base_fwd(c, &l);
  fa.img = x;
  fa.imgT = nullptr;
  fa.out32 = out;
  fa.out_stride = (size_t)n_ids * c->R;
  HIP_TRY(launch_forward(fa, c->st));
  return SLIM_OK;
}

slim_status slim_project_noalloc(slim_ctx* c, const int32_t* ids, int n_ids, const float* x,
                                 float* out) {
  if (!c) return fail(SLIM_EINVAL, "ctx is NULL");
  slim_status s = check_ids(c, ids, n_ids, true);
  if (s != SLIM_OK) return s;
  if (!x || !out) return fail(SLIM_EINVAL, "x and out must be non-NULL");
  const AngleList l = make_list(ids, n_ids);
  const size_t need = forward_partial_floats(c->h_geom.data(), c->N, c->R, l, c->B, c->tune_for(l.n));
  if (need > forward_scratch_floats())
    return fail(SLIM_EINVAL, "projection needs " + std::to_string(need) +
                                 " floats of scratch; the fixed scratch holds " +
                                 std::to_string(forward_scratch_floats()) + " (use slim_project)");
  float* scratch = forward_scratch(c->dev);
  if (!scratch) return fail(SLIM_EDEVICE, "fixed scratch not set up on this device");
  // the same launches as slim_project; every partial sum the reduction reads
  // is written first by the band kernel, so nothing is cleared
  FwdArgs fa = base_fwd(c, &l);
  fa.partial = scratch;
  fa.img = x;
  fa.imgT = nullptr;
  fa.out32 = out;
  fa.out_stride = (size_t)n_ids * c->R;
  HIP_TRY(launch_forward(fa, c->st));
  return SLIM_OK;
}

slim_status slim_backproject(slim_ctx* c, const int32_t* ids, int n_ids, const float* v, float* out) {
  if (!c) return fail(SLIM_EINVAL, "ctx is NULL");
  slim_status s = check_ids(c, ids, n_ids, true);
  if (s != SLIM_OK) return s;
  if (!v || !out) return fail(SLIM_EINVAL, "v and out must be non-NULL");
  const AngleList l = make_list(ids, n_ids);
  BackArgs ba;
  ba.tune = c->tune_for(l.n);
  ba.geom = c->d_geom;
  ba.N = c->N;
  ba.R = c->R;
  ba.B = c->B;
  ba.ids = &l;
  ba.v32 = v;
  ba.v_stride = (size_t)n_ids * c->R;
  ba.out = out;
  ba.img_stride = c->img_elems();
  ba.mode = 0;
  HIP_TRY(launch_back(ba, c->st));
  return SLIM_OK;
}

slim_status slim_data_backprojection(slim_ctx* c, const int32_t* ids, int n_ids, float* out) {
  if (!c) return fail(SLIM_EINVAL, "ctx is NULL");
  slim_status s = check_ids(c, ids, n_ids, false);
  if (s != SLIM_OK) return s;
  if (!out) return fail(SLIM_EINVAL, "out is NULL");
  if (!c->bound) return fail(SLIM_ESTATE, "no data bound (slim_set_data)");
  const AngleList l = make_list(ids, n_ids);
  const size_t need = (size_t)c->B * n_ids * c->R;
  if (need > c->gather_cap) {
    HIP_TRY(hipStreamSynchronize(c->st));
    HIP_TRY(hipFree(c->d_gather));
    c->d_gather = nullptr;
    c->gather_cap = 0;
    if (hipMalloc((void**)&c->d_gather, need * sizeof(float)) != hipSuccess)
      return fail(SLIM_ENOMEM, "gather workspace does not fit");
    c->gather_cap = need;
  }
  HIP_TRY(launch_gather_rows(c->b, c->bf16() ? 1 : 0, c->n_angles, c->R, c->B, l, c->d_gather,
                             c->st));
  BackArgs ba;
  ba.tune = c->tune_for(l.n);
  ba.geom = c->d_geom;
  ba.N = c->N;
  ba.R = c->R;
  ba.B = c->B;
  ba.ids = &l;
  ba.v32 = c->d_gather;
  ba.v_stride = (size_t)n_ids * c->R;
  ba.out = out;
  ba.img_stride = c->img_elems();
  ba.mode = 0;
  HIP_TRY(launch_back(ba, c->st));
  return SLIM_OK;
}

slim_status slim_warmstart(slim_ctx* c, slim_cnn* net, const int32_t* ids, int n_ids, float* x0,
                           int* used_net) {
  if (used_net) *used_net = 0;
  if (!c) return fail(SLIM_EINVAL, "ctx is NULL");
  slim_status s = check_ids(c, ids, n_ids, false);
  if (s != SLIM_OK) return s;
  if (!x0) return fail(SLIM_EINVAL, "x0 is NULL");
  if (!c->bound) return fail(SLIM_ESTATE, "no data bound (slim_set_data)");
  if (net && cnn_side(net) != c->N) return fail(SLIM_EINVAL, "network image size differs from N");
  const size_t nimg = c->img_elems() * c->B;
  // x0 may be the bound image: then the iteration restarts from it, with the
  // projectors' copies of x refreshed
  auto restart = [&]() -> slim_status {
    if (x0 != c->x) return SLIM_OK;
    c->k = 0;
    c->norms_valid = false;
    c->window.clear();
    c->epoch = 0;
    c->pos = 0;
    c->total_pcg_iters = 0;
    return transpose_slices(c);
  };
  if (!cnn_usable(net)) {
    HIP_TRY(hipMemsetAsync(x0, 0, nimg * sizeof(float), c->st));
    return restart();
  }
  s = slim_data_backprojection(c, ids, n_ids, c->d_tmp);
  if (s != SLIM_OK) return s;
  const int mb = cnn_max_batch(net);
  for (int b0 = 0; b0 < c->B; b0 += mb) {
    const int nb = std::min(mb, c->B - b0);
    s = cnn_forward_on(net, c->d_tmp + (size_t)b0 * c->img_elems(),
                       x0 + (size_t)b0 * c->img_elems(), nb, c->st);
    if (s != SLIM_OK) return s;
  }
  if (used_net) *used_net = 1;
  return restart();
}

slim_status slim_gram(slim_ctx* c, const int32_t* ida, int na, const int32_t* idb, int nb, double* out) {
  if (!c) return fail(SLIM_EINVAL, "ctx is NULL");
  slim_status s = check_ids(c, ida, na, true);
  if (s != SLIM_OK) return s;
  s = check_ids(c, idb, nb, true);
  if (s != SLIM_OK) return s;
  if (!out) return fail(SLIM_EINVAL, "out is NULL");
  HIP_TRY(launch_gram(c->d_geom, c->N, c->R, make_list(ida, na), make_list(idb, nb), out,
                      (int64_t)nb * c->R, c->st));
  return SLIM_OK;
}

// State blob: magic, k, epoch, pos, window size, then g ids per window block.
slim_status slim_get_state(slim_ctx* c, void* buf, int64_t* size) {
  if (!c || !size) return fail(SLIM_EINVAL, "ctx or size is NULL");
  const int64_t need = (int64_t)sizeof(int32_t) * (5 + c->window.size() * c->g);
  if (!buf || *size < need) {
    *size = need;
    return fail(SLIM_EINVAL, "state buffer too small");
  }
  int32_t* w = (int32_t*)buf;
  w[0] = 0x534c494d;
  w[1] = c->k;
  w[2] = c->epoch;
  w[3] = c->pos;
  w[4] = (int32_t)c->window.size();
  int q = 5;
  for (int s : c->window)
    for (int a : c->slot_ids[s]) w[q++] = a;
  *size = need;
  return SLIM_OK;
}

slim_status slim_set_state(slim_ctx* c, const void* buf, int64_t size) {
  if (!c || !buf) return fail(SLIM_EINVAL, "ctx or buf is NULL");
  if (!c->bound) return fail(SLIM_ESTATE, "bind data before restoring state");
  const int32_t* w = (const int32_t*)buf;
  if (size < (int64_t)sizeof(int32_t) * 5 || w[0] != 0x534c494d) return fail(SLIM_ESTATE, "bad state blob");
  const int W = w[4];
  if (W < 0 || W > c->r + 1 || size < (int64_t)sizeof(int32_t) * (5 + W * c->g) || w[1] < W)
    return fail(SLIM_ESTATE, "bad state blob");
  for (int i = 0; i < W * c->g; ++i)
    if (w[5 + i] < 0 || w[5 + i] >= c->n_angles) return fail(SLIM_ESTATE, "bad angle id in state");
  c->k = w[1] - W;
  c->window.clear();
  c->epoch = w[2];
  c->pos = w[3];
  // replay the window's block entries without touching x: refill slots in
  // the order the original run filled them, so slot numbers match
  const int S = c->r + 1;
  for (int i = 0; i < W; ++i) {
    const int slot = c->k % S;
    if ((int)c->window.size() == S) c->window.pop_front();
    c->slot_ids[slot].assign(w + 5 + i * c->g, w + 5 + (i + 1) * c->g);
    c->window.push_back(slot);
    if (c->mode == SLIM_GRAM_CHOL) {
      AngleList na = make_list(c->slot_ids[slot].data(), c->g);
      for (int q : c->window) {
        AngleList nb = make_list(c->slot_ids[q].data(), c->g);
        double* T = c->d_tiles + ((int64_t)slot * S + q) * c->ell * c->ell;
        HIP_TRY(launch_gram(c->d_geom, c->N, c->R, na, nb, T, c->ell, c->st));
      }
    }
    c->k += 1;
  }
  HIP_TRY(transpose_slices(c) == SLIM_OK ? hipSuccess : hipErrorUnknown);
  return SLIM_OK;
}

slim_status slim_slice_norms(slim_ctx* c, double* out, int n) {
  if (!c || !out) return fail(SLIM_EINVAL, "ctx or out is NULL");
  if (n != c->B) return fail(SLIM_EINVAL, "n must equal n_slices");
  if (!c->norms_valid) return fail(SLIM_ESTATE, "no step read back since the data were bound");
  for (int sl = 0; sl < c->B; ++sl) {
    out[3 * sl + 0] = std::sqrt(c->h_norms[3 * sl + 0]);
    out[3 * sl + 1] = std::sqrt(c->h_norms[3 * sl + 1]);
    out[3 * sl + 2] = c->x_true ? std::sqrt(c->h_norms[3 * sl + 2]) : -1.0;
  }
  return SLIM_OK;
}


// ------------------------------------------------------------- autotuner
}  // extern "C"

namespace {

struct TuneEntry {
  ProjTune tune;
  slim_tune_info info;
};
std::mutex g_tune_mu;
std::map<std::tuple<int, int, int, int>, TuneEntry> g_tune_cache;

bool valid_tune(const slim_tune& t) {
  auto in = [](int v, std::initializer_list<int> ok) {
    for (int o : ok)
      if (v == o) return true;
    return false;
  };
  return in(t.fwd_bt, {0, 1, 2, 4}) && in(t.fwd_items, {0, 2, 3, 4, 6, 8, 10}) &&
         in(t.fwd_slots, {0, 2, 4}) && in(t.back_bt, {0, 1, 2, 4});
}

ProjTune to_proj(const slim_tune& t) {
  ProjTune p;
  p.fwd_bt = t.fwd_bt;
  p.fwd_items = t.fwd_items;
  p.fwd_slots = t.fwd_slots;
  p.back_bt = t.back_bt;
  return p;
}

slim_tune to_public(const ProjTune& p) {
  slim_tune t;
  t.fwd_bt = p.fwd_bt;
  t.fwd_items = p.fwd_items;
  t.fwd_slots = p.fwd_slots;
  t.back_bt = p.back_bt;
  return t;
}

}  // namespace

extern "C" {

slim_status slim_set_tune(slim_ctx* c, const slim_tune* t) {
  if (!c || !t) return fail(SLIM_EINVAL, "ctx or tune is NULL");
  if (!valid_tune(*t)) return fail(SLIM_EINVAL, "tune field outside its allowed values");
  c->tune = to_proj(*t);
  c->tune_by_n.clear();
  return SLIM_OK;
}

slim_status slim_get_tune(slim_ctx* c, slim_tune* t) {
  if (!c || !t) return fail(SLIM_EINVAL, "ctx or tune is NULL");
  *t = to_public(c->tune);
  return SLIM_OK;
}

slim_status slim_autotune(slim_ctx* c, int n_ids, int force, slim_tune_info* info) {
  if (!c) return fail(SLIM_EINVAL, "ctx is NULL");
  if (n_ids < 0 || n_ids > std::min(kMaxList, c->n_angles))
    return fail(SLIM_EINVAL, "n_ids must be in [0, min(256, n_angles)]");
  AngleList lists[2];
  int nlists = 1;
  lists[0].n = lists[1].n = 0;
  AngleList& win = lists[0];
  const bool window = n_ids == 0;
  if (window) {  // the CG window: r+1 blocks spread over [0, pi)
    const int M = c->n_angles / c->g;
    const int nblk = std::min(c->r + 1, M);
    for (int j = 0; j < nblk; ++j) {
      const int beta = (int)((int64_t)j * M / nblk);
      for (int a = 0; a < c->g; ++a) win.id[win.n++] = beta * c->g + a;
    }
  } else {       // a block of n_ids adjacent angles from 0 and from pi/2
    nlists = 2 * n_ids <= c->n_angles ? 2 : 1;
    for (int L = 0; L < nlists; ++L)
      for (int j = 0; j < n_ids; ++j) lists[L].id[lists[L].n++] = L * (c->n_angles / 2) + j;
  }
  for (int L = 0; L < 2; ++L)
    for (int i = lists[L].n; i < kMaxList; ++i) lists[L].id[i] = 0;
  auto keep = [&](const ProjTune& t) {
    c->tune_by_n[win.n] = t;
    if (window) c->tune = t;
  };
  const auto key = std::make_tuple(c->N, c->B, c->R, win.n);
  if (!force) {
    std::lock_guard<std::mutex> lk(g_tune_mu);
    auto it = g_tune_cache.find(key);
    if (it != g_tune_cache.end()) {
      keep(it->second.tune);
      if (info) {
        *info = it->second.info;
        info->cached = 1;
      }
      return SLIM_OK;
    }
  }

  // candidate shapes; the built-in rules first
  std::vector<ProjTune> fwd_c(1), back_c(1);
  const int bt_max = slice_tile(c->B);
  for (int bt : {1, 2, 4}) {
    if (bt > bt_max) continue;
    ProjTune b;
    b.back_bt = bt;
    back_c.push_back(b);
    for (int it : {2, 3, 4, 6, 8}) {
      if (it > forward_max_items(bt)) continue;
      for (int sl : {2, 4}) {
        ProjTune f;
        f.fwd_bt = bt;
        f.fwd_items = it;
        f.fwd_slots = sl;
        fwd_c.push_back(f);
      }
    }
  }
  size_t part = 0;
  for (int L = 0; L < nlists; ++L)
    for (const ProjTune& t : fwd_c)
      part = std::max(part, forward_partial_floats(c->h_geom.data(), c->N, c->R, lists[L], c->B, t));

  // workspace: an image and its transpose (zeros), the window's rays, partials
  const size_t nimg = c->img_elems() * c->B;
  const size_t nray = (size_t)c->B * win.n * c->R;
  float *img = nullptr, *imgT = nullptr, *rays = nullptr, *fpart = nullptr;
  hipEvent_t e0 = nullptr, e1 = nullptr;
  auto release = [&]() {
    (void)hipFree(img);
    (void)hipFree(imgT);
    (void)hipFree(rays);
    (void)hipFree(fpart);
    if (e0) (void)hipEventDestroy(e0);
    if (e1) (void)hipEventDestroy(e1);
  };
  HIP_TRY(hipStreamSynchronize(c->st));
  if (hipMalloc((void**)&img, nimg * sizeof(float)) != hipSuccess ||
      hipMalloc((void**)&imgT, nimg * sizeof(float)) != hipSuccess ||
      hipMalloc((void**)&rays, nray * sizeof(float)) != hipSuccess ||
      hipMalloc((void**)&fpart, part * sizeof(float)) != hipSuccess) {
    release();
    return fail(SLIM_ENOMEM, "autotune workspace does not fit");
  }
  hipError_t e = hipSuccess;
  if (e == hipSuccess) e = hipMemsetAsync(img, 0, nimg * sizeof(float), c->st);
  if (e == hipSuccess) e = hipMemsetAsync(imgT, 0, nimg * sizeof(float), c->st);
  if (e == hipSuccess) e = hipMemsetAsync(rays, 0, nray * sizeof(float), c->st);
  if (e == hipSuccess) e = hipEventCreate(&e0);
  if (e == hipSuccess) e = hipEventCreate(&e1);
  if (e != hipSuccess) {
    release();
    return fail(SLIM_EDEVICE, std::string("autotune: ") + hipGetErrorString(e));
  }
  // mean time of 3 launches after one warm-up launch, microseconds
  auto timed = [&](auto&& launch, double* us) -> hipError_t {
    hipError_t r = launch();
    if (r != hipSuccess) return r;
    if ((r = hipEventRecord(e0, c->st)) != hipSuccess) return r;
    for (int k = 0; k < 3; ++k)
      if ((r = launch()) != hipSuccess) return r;
    if ((r = hipEventRecord(e1, c->st)) != hipSuccess) return r;
    if ((r = hipEventSynchronize(e1)) != hipSuccess) return r;
    float ms = 0.f;
    if ((r = hipEventElapsedTime(&ms, e0, e1)) != hipSuccess) return r;
    *us = ms * 1e3 / 3.0;
    return hipSuccess;
  };
  slim_tune_info ti{};
  // every candidate is timed in kRounds interleaved rounds and scored by its
  // fastest round (clock and cache drift then affect all candidates alike)
  constexpr int kRounds = 3;
  std::vector<double> tf(fwd_c.size(), 1e300), tb(back_c.size(), 1e300);
  for (int round = 0; round < kRounds && e == hipSuccess; ++round) {
    for (size_t k = 0; k < fwd_c.size() && e == hipSuccess; ++k) {
      double sum = 0.0;
      for (int L = 0; L < nlists && e == hipSuccess; ++L) {
        FwdArgs fa;
        fa.tune = fwd_c[k];
        fa.geom = c->d_geom;
        fa.h_geom = c->h_geom.data();
        fa.N = c->N;
        fa.R = c->R;
        fa.B = c->B;
        fa.ids = &lists[L];
        fa.img = img;
        fa.imgT = imgT;
        fa.img_stride = c->img_elems();
        fa.out32 = rays;
        fa.out_stride = (size_t)win.n * c->R;
        fa.partial = fpart;
        double us = 0.0;
        e = timed([&]() { return launch_forward(fa, c->st); }, &us);
        sum += us;
      }
      tf[k] = std::min(tf[k], sum);
    }
    for (size_t k = 0; k < back_c.size() && e == hipSuccess; ++k) {
      double sum = 0.0;
      for (int L = 0; L < nlists && e == hipSuccess; ++L) {
        BackArgs ba;
        ba.tune = back_c[k];
        ba.geom = c->d_geom;
        ba.N = c->N;
        ba.R = c->R;
        ba.B = c->B;
        ba.ids = &lists[L];
        ba.v32 = rays;
        ba.v_stride = (size_t)win.n * c->R;
        ba.out = img;
        ba.img_stride = c->img_elems();
        ba.mode = 0;
        double us = 0.0;
        e = timed([&]() { return launch_back(ba, c->st); }, &us);
        sum += us;
      }
      tb[k] = std::min(tb[k], sum);
    }
  }
  double best_f = 1e300, best_b = 1e300;
  ProjTune best;
  for (size_t k = 0; k < fwd_c.size(); ++k)
    if (tf[k] < best_f) {
      best_f = tf[k];
      best.fwd_bt = fwd_c[k].fwd_bt;
      best.fwd_items = fwd_c[k].fwd_items;
      best.fwd_slots = fwd_c[k].fwd_slots;
    }
  for (size_t k = 0; k < back_c.size(); ++k)
    if (tb[k] < best_b) {
      best_b = tb[k];
      best.back_bt = back_c[k].back_bt;
    }
  ti.fwd_default_us = tf[0];
  ti.back_default_us = tb[0];
  release();
  if (e != hipSuccess) return fail(SLIM_EDEVICE, std::string("autotune: ") + hipGetErrorString(e));
  ti.chosen = to_public(best);
  ti.fwd_us = best_f;
  ti.back_us = best_b;
  ti.candidates = (int)(fwd_c.size() + back_c.size());
  ti.cached = 0;
  keep(best);
  {
    std::lock_guard<std::mutex> lk(g_tune_mu);
    g_tune_cache[key] = TuneEntry{best, ti};
  }
  if (info) *info = ti;
  return SLIM_OK;
}

slim_status slim_profile(slim_ctx* c, int on) {
  if (!c) return fail(SLIM_EINVAL, "ctx is NULL");
  HIP_TRY(hipStreamSynchronize(c->st));
  if (c->prof.on) HIP_TRY(c->prof.harvest());
  c->prof.on = on != 0;
  for (int k = 0; k < K_COUNT; ++k) {
    c->prof.total_ms[k] = 0.0;
    c->prof.launches[k] = 0;
  }
  return SLIM_OK;
}

slim_status slim_kernel_stats(slim_ctx* c, int kind, double* total_ms, int64_t* launches) {
  if (!c || !total_ms || !launches) return fail(SLIM_EINVAL, "NULL argument");
  if (kind < 0 || kind >= K_COUNT) return fail(SLIM_EINVAL, "unknown kernel kind");
  HIP_TRY(hipStreamSynchronize(c->st));
  if (c->prof.on) HIP_TRY(c->prof.harvest());
  *total_ms = c->prof.total_ms[kind];
  *launches = c->prof.launches[kind];
  return SLIM_OK;
}

void slim_destroy(slim_ctx* c) {
  if (!c) return;
  (void)hipStreamSynchronize(c->st);
  delete c;
}

}  // extern "C"

// ------------------------------------------------------------------ groups
struct slim_group {
  std::vector<slim_ctx*> ctx;
  bool grouped = false;            // CG solves in shared launches
  PcgGroupWork gw;                 // their descriptor tables and graph
  std::vector<hipEvent_t> ev;      // one per context: hand-over between streams
  ~slim_group() {
    pcg_group_free(gw);
    for (hipEvent_t e : ev)
      if (e) (void)hipEventDestroy(e);
  }
};

namespace {

// The group's CG solves (contexts in CG mode with a solve in progress) in
// shared launches on the first such context's stream: the other contexts'
// streams hand their work over by events before, and take it back after.
slim_status group_cg_shared(slim_group* g, StepState* ss, const std::vector<int>& idx) {
  const int m = (int)idx.size();
  hipStream_t st0 = g->ctx[idx[0]]->st;
  for (int j = 1; j < m; ++j) {
    slim_ctx* c = g->ctx[idx[j]];
    HIP_TRY(hipEventRecord(g->ev[idx[j]], c->st));
    HIP_TRY(hipStreamWaitEvent(st0, g->ev[idx[j]], 0));
  }
  PcgRun* runs[kMaxGroup];
  bool graphs = true;
  for (int j = 0; j < m; ++j) {
    runs[j] = &ss[idx[j]].run;
    graphs = graphs && g->ctx[idx[j]]->graphs();
  }
  PcgGroupRun gr;
  hipError_t e = pcg_group_begin(gr, g->gw, runs, m, st0);
  while (e == hipSuccess && !gr.done) {
    e = pcg_group_enqueue(gr, graphs);
    if (e == hipSuccess) e = pcg_group_poll(gr);
  }
  if (e != hipSuccess) return fail(SLIM_EDEVICE, std::string("grouped CG: ") + hipGetErrorString(e));
  for (int j = 0; j < m; ++j) runs[j]->done = true;
  HIP_TRY(hipEventRecord(g->ev[idx[0]], st0));
  for (int j = 1; j < m; ++j) HIP_TRY(hipStreamWaitEvent(g->ctx[idx[j]]->st, g->ev[idx[0]], 0));
  return SLIM_OK;
}

}  // namespace

extern "C" {

slim_status slim_group_create(slim_group** out, slim_ctx* const* ctxs, int n) {
  if (!out || !ctxs || n < 1) return fail(SLIM_EINVAL, "out or ctxs is NULL, or n < 1");
  *out = nullptr;
  for (int i = 0; i < n; ++i) {
    if (!ctxs[i]) return fail(SLIM_EINVAL, "a context is NULL");
    for (int j = 0; j < i; ++j)
      if (ctxs[j] == ctxs[i]) return fail(SLIM_EINVAL, "a context is listed twice");
    if (ctxs[i]->n_angles != ctxs[0]->n_angles || ctxs[i]->g != ctxs[0]->g)
      return fail(SLIM_EINVAL, "contexts differ in n_angles or angles_per_block");
  }
  slim_group* g = new slim_group;
  g->ctx.assign(ctxs, ctxs + n);
  g->ev.assign(n, nullptr);
  hipError_t e = hipSuccess;
  for (int i = 0; i < n && e == hipSuccess; ++i)
    e = hipEventCreateWithFlags(&g->ev[i], hipEventDisableTiming);
  if (e == hipSuccess && n <= kMaxGroup) e = pcg_group_alloc(g->gw, n);
  g->grouped = false;
  if (e != hipSuccess) {
    delete g;
    return fail(SLIM_EDEVICE, std::string("group: ") + hipGetErrorString(e));
  }
  *out = g;
  return SLIM_OK;
}

slim_status slim_group_set_shared(slim_group* g, int on) {
  if (!g) return fail(SLIM_EINVAL, "group is NULL");
  if (on != 0 && on != 1) return fail(SLIM_EINVAL, "on must be 0 or 1");
  if (on && g->ctx.size() > (size_t)kMaxGroup)
    return fail(SLIM_EINVAL, "shared launches hold at most 16 contexts");
  g->grouped = on != 0;
  return SLIM_OK;
}

slim_status slim_group_step(slim_group* g, const int32_t* ids, int n_ids, slim_step_info* infos) {
  if (!g) return fail(SLIM_EINVAL, "group is NULL");
  const int n = (int)g->ctx.size();
  for (slim_ctx* c : g->ctx) {
    if (n_ids != c->g) return fail(SLIM_EINVAL, "n_ids must equal angles_per_block");
    slim_status s = check_ids(c, ids, n_ids, false);
    if (s != SLIM_OK) return s;
    if (!c->bound) return fail(SLIM_ESTATE, "no data bound (slim_set_data)");
    if (c->streaming)
      return fail(SLIM_ESTATE, "streaming context: step it with slim_step_data, not in a group");
  }
  std::unique_ptr<StepState[]> ss(new StepState[n]);  // fixed addresses (CG runs)
  // every context's fallible host work first, so that a refused step leaves
  // all of them as they were
  for (int i = 0; i < n; ++i) {
    std::deque<int> win;
    plan_window(g->ctx[i], ids, ss[i], win);
    slim_status s = step_prepare(g->ctx[i], ss[i]);
    if (s != SLIM_OK) return s;
  }
  auto unbind_all = [&]() {
    for (slim_ctx* c : g->ctx) c->bound = false;
  };
  for (int i = 0; i < n; ++i) {
    slim_status s = step_begin(g->ctx[i], ids, ss[i]);
    if (s != SLIM_OK) {
      unbind_all();
      return s;
    }
  }
  {
    std::vector<int> cg;
    bool profiling = false;
    for (int i = 0; i < n; ++i) {
      if (ss[i].pcg && !ss[i].run.done) cg.push_back(i);
      profiling = profiling || g->ctx[i]->prof.on;
    }
    // shared launches for two or more solves (kernel timing keeps the
    // contexts' own launches, which its counters follow)
    if (g->grouped && cg.size() >= 2 && !profiling) {
      slim_status s = group_cg_shared(g, ss.get(), cg);
      if (s != SLIM_OK) {
        unbind_all();
        return s;
      }
    }
  }
  for (bool all = false; !all;) {
    all = true;
    for (int i = 0; i < n; ++i)
      if (ss[i].pcg && !ss[i].run.done) {
        hipError_t e = pcg_enqueue(ss[i].run, g->ctx[i]->graphs());
        if (e != hipSuccess) {
          unbind_all();
          return fail(SLIM_EDEVICE, std::string("pcg: ") + hipGetErrorString(e));
        }
      }
    for (int i = 0; i < n; ++i)
      if (ss[i].pcg && !ss[i].run.done) {
        hipError_t e = pcg_poll(ss[i].run);
        if (e != hipSuccess) {
          unbind_all();
          return fail(SLIM_EDEVICE, std::string("pcg: ") + hipGetErrorString(e));
        }
        all = all && ss[i].run.done;
      }
  }
  slim_status first = SLIM_OK;
  for (int i = 0; i < n; ++i) {
    slim_status s = step_end(g->ctx[i], ss[i], infos ? infos + i : nullptr);
    if (s == SLIM_EDEVICE) g->ctx[i]->bound = false;
    if (s != SLIM_OK && first == SLIM_OK) first = s;
  }
  return first;
}

void slim_group_destroy(slim_group* g) { delete g; }

}  // extern "C"
