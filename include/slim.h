/*
 * slim.h -- C ABI of the MI355X (gfx950) slimLS library.
 *
 * slimLS (Chung, Chung, Slagel, Tenorio, arXiv 1912.07962, sec. 1,
 * eq. (ram) and eq. (B_k)) iterates
 *
 *     x_k = x_{k-1} - (lambda I + M_k^T M_k)^{-1} A_k^T (A_k x_{k-1} - b_k),
 *     M_k = [A_{k-r}; ...; A_k]        (C_k = I, alpha_k = 1/lambda),
 *
 * where A_k is a sampled block of rows of A.  Here A is the 2D parallel-beam
 * projector of an N x N image (sec. 4.3 experiments) and a block is a set of
 * projection angles.  The library evaluates A matrix-free with Joseph
 * weights
 *     a[(theta,s),(i,j)] = (h/d) max(0, 1 - |s - x_j cos - y_i sin| / (h d)),
 *     d = max(|cos|, |sin|), h = 2/N,
 * pixel centres x_j = (j-(N-1)/2) h, y_i = (i-(N-1)/2) h (row i, column j,
 * row-major), ray offsets s_t = (t-(R-1)/2) h.  The step is computed in the
 * Gram (push-through) form s = M^T z, (M M^T + lambda I) z = [0;...;0;res],
 * by FP64 Cholesky of the explicit Gram, or by preconditioned CG on the same
 * system when p = rows(M) is large.
 *
 * Conventions for every entry point:
 *  - Array arguments marked "device" are device pointers (e.g. from torch
 *    tensors); "host" arrays are ordinary host memory.  The caller owns all
 *    arrays; the library only borrows them for the duration of a call (and,
 *    for slim_set_data, until the next slim_set_data or slim_destroy).
 *  - Layouts: image [n_slices][N][N] float32, row-major; sinogram
 *    [n_slices][n_angles][n_rays] float32 (bf16 when precision is
 *    SLIM_PREC_BF16, see slim_opts), angle-major.
 *  - Work is enqueued on opts.stream (a hipStream_t; NULL is the default
 *    stream).  Calls that return host-visible numbers (step info, solve info)
 *    synchronise that stream.
 *  - No entry point throws; every error is a slim_status.  Argument checks
 *    happen before any device work.  A context is bound to one device and
 *    one stream and is not thread-safe.
 */
#ifndef SLIM_H
#define SLIM_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
  SLIM_OK = 0,
  SLIM_EINVAL = 1,   /* invalid argument (message via slim_last_error)        */
  SLIM_ENOMEM = 2,   /* device workspace does not fit                         */
  SLIM_EDEVICE = 3,  /* a HIP call failed                                     */
  SLIM_ENUMERIC = 4, /* non-finite norm or non-positive Cholesky pivot        */
  SLIM_ENOTCONV = 5, /* CG reached its iteration cap (the step is still taken) */
  SLIM_ESTATE = 6    /* step/solve before slim_set_data, or bad state blob    */
} slim_status;

typedef struct slim_ctx slim_ctx;

typedef struct {
  int N;        /* pixels per side, >= 2                                  */
  int n_slices; /* independent slices sharing A (1 for a single image)    */
} slim_grid;

enum { SLIM_PREC_FP32 = 0, SLIM_PREC_BF16 = 1 };
/* Gram solve: AUTO (2D: Cholesky while p <= chol_max_p, else CG; 3D:
 * Jacobi-preconditioned CG), CHOL (2D only), PCG (plain CG), JACOBI (3D
 * only: CG preconditioned by the inverse of the Gram diagonal). */
enum { SLIM_GRAM_AUTO = 0, SLIM_GRAM_CHOL = 1, SLIM_GRAM_PCG = 2, SLIM_GRAM_JACOBI = 3 };

typedef struct {
  int angles_per_block; /* g: angles in one sampled block; divides n_angles */
  int precision;        /* SLIM_PREC_FP32 or SLIM_PREC_BF16 (bf16 sinogram
                           input and bf16 image shadow read by the forward
                           projector; fp32 master image and accumulation)  */
  int gram_mode;        /* SLIM_GRAM_AUTO / CHOL / PCG / JACOBI             */
  int chol_max_p;       /* AUTO uses Cholesky while p <= chol_max_p         */
  int pcg_max_iter;     /* CG iteration cap per step                        */
  double pcg_tol;       /* CG stop: ||res|| <= pcg_tol * ||rhs||            */
  int check_every;      /* slim_solve: read the step norms every q steps    */
  uint64_t seed;        /* slim_solve: SplitMix64 seed of the block order   */
  void* stream;         /* hipStream_t work queue (NULL = default stream)   */
  int use_graph;        /* 1: the 8-iteration chunks of a step's CG after
                           the first are replayed from one hipGraph, captured
                           while the first chunk runs (only on a stream other
                           than NULL, and not while kernel timing is on;
                           short chunks near the stop are launched directly);
                           0: launched one by one                          */
  int damping_ramp;     /* 1: ramped damping of sec. 4.2 (used in sec. 4.3):
                           alpha_k = k alpha / (r+1) for the first r+1 steps,
                           i.e. step k uses lambda (r+1) / k while k <= r and
                           lambda after; 0: constant lambda                */
  double tikhonov;      /* > 0: slimTik (sec. 2, eq. (slimTik)) with L = I,
                           the Tikhonov parameter of eq. (TLS1): each step
                           solves ((lambda_k + W t^2/M) I + M^T M) s =
                           A_k^T res + (t^2/M) x_{k-1}, W the blocks in the
                           window, M = n_angles / g (the printed equation
                           has r t^2/M; W = r+1 once the window is full is
                           what slimLS on the stacked rows [A_k; t/sqrt(M) I]
                           gives).  Costs one more forward projection of the
                           window per step.  FP32 precision only.
                           0: plain slimLS                                  */
} slim_opts;

typedef struct {
  double step_norm; /* ||s_k||_2 (max over slices when n_slices > 1)        */
  double x_norm;    /* ||x_k||_2 (of the slice attaining step_norm)         */
  double err_norm;  /* ||x_k - x_true||_2, or -1 without x_true             */
  int k;            /* iteration count after this step                      */
  int pcg_iters;    /* CG iterations of this step (0 in Cholesky mode)      */
  double pcg_relres;/* final CG relative residual (0 in Cholesky mode)      */
} slim_step_info;

typedef struct {
  int steps;        /* steps taken                                          */
  int epochs;       /* epochs started                                       */
  int converged;    /* 1 if the stop rule fired                             */
  double rho_last;  /* last ||s_k|| / ||x_k|| read                          */
  double err_last;  /* last ||x_k - x_true|| / ||x_true|| (-1 if unknown)   */
  int pcg_iters;    /* total CG iterations                                  */
} slim_solve_info;

/* Fill *opts with defaults: g = 1, FP32, AUTO, chol_max_p = 8192,
 * pcg_max_iter = 1000, pcg_tol = 1e-6, check_every = 1, seed = 0, NULL stream,
 * use_graph = 1, damping_ramp = 0, tikhonov = 0. */
slim_status slim_default_opts(slim_opts* opts);

/* Create a context (paper sec. 1 setup, sec. 4.3 geometry).
 *  grid      host; 2 <= N <= 8192, n_slices >= 1
 *  n_angles  number of projection angles (>= 1)
 *  angles    host [n_angles] radians in [0, pi), or NULL for a*pi/n_angles
 *  n_rays    rays per angle, 1 <= R <= 4096 (spacing h, centred on the axis)
 *  r         memory level r >= 0 (sec. 1, eq. (B_k))
 *  lambda    damping 1/alpha > 0, finite
 *  opts      host, or NULL for defaults
 * Allocates the geometry table and all step workspace on the current device.
 * Errors: SLIM_EINVAL (checked before any device call), SLIM_ENOMEM, SLIM_EDEVICE. */
slim_status slim_init(slim_ctx** out, const slim_grid* grid, int n_angles, const double* angles,
                      int n_rays, int r, double lambda, const slim_opts* opts);

/* Bind the data of the problem b = A x_true + eps (sec. 1, eq. (inverseproblem)).
 *  b       device sinogram [n_slices][n_angles][n_rays] (float32, or bf16 bits
 *          when precision is SLIM_PREC_BF16), or NULL for streaming data: each
 *          block's rows then arrive with its step (slim_step_data) and are kept
 *          in a sinogram the library allocates (rows not yet delivered are
 *          zero, also for slim_data_backprojection and slim_warmstart)
 *  x       device image [n_slices][N][N] float32: the iterate, read and
 *          overwritten in place by slim_step / slim_solve
 *  x_true  device [n_slices][N][N] float32 or NULL; enables err_norm
 * Resets the iteration (k = 0, empty memory window).
 * Errors: SLIM_EINVAL on NULL x; SLIM_ENOMEM, SLIM_EDEVICE (streaming buffers). */
slim_status slim_set_data(slim_ctx* ctx, const void* b, void* x, const float* x_true);

/* One slimLS iteration (eq. (ram)) with the sampled block A_k = rows of the
 * given angles (host int32 [n_ids], n_ids == angles_per_block, each in
 * [0, n_angles), no duplicates).  The block enters the memory window; the
 * oldest block leaves once the window holds r+1 blocks.  info may be NULL
 * (then nothing is read back and the stream is not synchronised).
 * Errors: SLIM_EINVAL (bad ids), SLIM_ESTATE (no data), SLIM_ENOMEM (the
 * projector's workspace for this window does not fit; the step is not taken
 * and the context is unchanged), SLIM_ENUMERIC, SLIM_ENOTCONV (CG cap
 * reached; the step is still applied), SLIM_EDEVICE (the context is left
 * unbound: rebind with slim_set_data before the next step). */
slim_status slim_step(slim_ctx* ctx, const int32_t* angle_ids, int n_ids, slim_step_info* info);

/* slim_step for streaming data (data bound with b = NULL).  The method needs
 * a block's data only when the block is sampled (sec. 1, eq. (ram): only b_k
 * enters step k), so the caller passes it with the step:
 *  b_block  [n_slices][n_ids][n_rays] float32 (bf16 bits when SLIM_PREC_BF16),
 *           the rows of angle_ids in that order; host or device memory.  Device
 *           memory is read in the order of the context's stream; host memory is
 *           copied on a stream of the library's own (default priority) into one
 *           of two staging buffers, so the copy of step k+1 overlaps step k when
 *           the caller does not read step k back (info == NULL); use pinned
 *           host memory for the copy to run asynchronously, and keep b_block
 *           unchanged until the step's results are read or the context's stream
 *           is synchronised.
 * Errors: as slim_step; SLIM_EINVAL on NULL b_block; SLIM_ESTATE unless the
 * data were bound with b = NULL (and slim_step returns SLIM_ESTATE on such a
 * context). */
slim_status slim_step_data(slim_ctx* ctx, const int32_t* angle_ids, int n_ids,
                           const void* b_block, slim_step_info* info);

/* Set the damping lambda = 1/alpha used by the following steps (eq. (B_k)
 * with C_k = I).  The end of sec. 3 suggests a constant alpha_k for fast
 * initial progress, then a decaying alpha_k (a growing lambda) for accuracy;
 * the paper gives no formula for the decay, so the caller drives it by
 * calling this between steps.  With damping_ramp on, steps k <= r still use lambda (r+1) / k of
 * the value set here.  lambda is a parameter of the context, not of the
 * iteration state (slim_get_state does not hold it).
 * Errors: SLIM_EINVAL (NULL ctx, lambda not positive and finite). */
slim_status slim_set_lambda(slim_ctx* ctx, double lambda);

/* Per-slice norms of the last step whose info was read back (slim_step
 * with info != NULL, or slim_solve): out is host float64 [n_slices][3]
 * holding ||s_k||, ||x_k|| and ||x_k - x_true|| (-1 without x_true) of each
 * slice, the quantities of the stop rule (sec. 4.3) slice by slice.
 * Errors: SLIM_EINVAL (NULL out or n != n_slices), SLIM_ESTATE (no step read
 * back since the data were bound). */
slim_status slim_slice_norms(slim_ctx* ctx, double* out, int n);

/* Run slimLS from x (in: x0, out: the result) with the data b until the stop
 * rule or max_epochs.  Blocks are the fixed partition {g*beta, ..., g*beta+g-1}
 * of the angles, visited random-cyclically (sec. 4.3): epoch e visits every
 * block once in the order of a Fisher-Yates shuffle driven by SplitMix64
 * outputs e*(M-1)+1 ... e*(M-1)+(M-1) of opts.seed.  Stop rule: the first
 * k >= r+1 (checked every check_every steps) with ||s_k|| <= tol ||x_k||
 * (sec. 4.3 early termination); tol <= 0 runs all epochs.
 *  b, x, x_true as in slim_set_data (this call binds them).
 * Errors: as slim_set_data and slim_step. */
slim_status slim_solve(slim_ctx* ctx, const void* b, void* x, const float* x_true, double tol,
                       int max_epochs, slim_solve_info* info);

/* Forward projection of rows of A (sec. 4.2: function evaluations of A_k).
 *  angle_ids  host int32 [n_ids] (any order, repeats allowed)
 *  x          device [n_slices][N][N] float32
 *  out        device [n_slices][n_ids][n_rays] float32, out = A_ids x
 * Errors: SLIM_EINVAL, SLIM_EDEVICE. */
slim_status slim_project(slim_ctx* ctx, const int32_t* angle_ids, int n_ids, const float* x,
                         float* out);

/* slim_project for callers that cannot allocate device memory (code under
 * HIP graph capture, tight serving loops, harnesses that forbid hipMalloc):
 * the same projection, launches and results, but the projector's partial
 * sums live in a fixed scratch array of 16 MiB (4,194,304 floats) that the
 * library's code object holds on each device it runs on until the process
 * ends, instead of the context's workspace (which slim_project grows with
 * hipMalloc).  This call allocates nothing and frees nothing; the scratch's
 * device address is taken once per device by slim_init.
 *  angle_ids, x, out as in slim_project (caller-owned).
 * The scratch needed is what slim_project's workspace needs for the same
 * call: n_slices * G * n_ids * n_rays floats, G the number of groups of image
 * bands the launch splits the image into (G = 8 for 88 angles of one 1024^2
 * image, 1.02 M floats); a call that needs more returns SLIM_EINVAL and
 * launches nothing (slim_project has no such limit).
 * Every call on one device shares that device's scratch and leaves its
 * contents behind (each call overwrites every entry it reads), so calls that
 * overlap on one device -- from different streams or threads -- race; calls
 * ordered on one stream do not.
 * Errors: SLIM_EINVAL (bad arguments, scratch too small), SLIM_EDEVICE. */
slim_status slim_project_noalloc(slim_ctx* ctx, const int32_t* angle_ids, int n_ids,
                                 const float* x, float* out);

/* Back-projection, the exact adjoint of slim_project with the same weights.
 *  v    device [n_slices][n_ids][n_rays] float32
 *  out  device [n_slices][N][N] float32, out = A_ids^T v (overwritten)
 * Errors: SLIM_EINVAL, SLIM_EDEVICE. */
slim_status slim_backproject(slim_ctx* ctx, const int32_t* angle_ids, int n_ids, const float* v,
                             float* out);

/* Back-projection of the bound data for the listed angles:
 * out = A_ids^T b_ids for every slice (sec. 1: the first iterate from x0 = 0
 * is built from such products; the learned warm start reads it).
 *  angle_ids  host int32 [n_ids], no duplicates
 *  out        device [n_slices][N][N] float32 (overwritten)
 * Errors: SLIM_EINVAL, SLIM_ESTATE (no data bound), SLIM_EDEVICE. */
slim_status slim_data_backprojection(slim_ctx* ctx, const int32_t* angle_ids, int n_ids,
                                     float* out);

/* Gram block A_ids_a A_ids_b^T (sec. 2 Woodbury remark; the blocks of
 * M_k M_k^T).  out: device float64 [n_a*n_rays][n_b*n_rays], row-major.
 * Errors: SLIM_EINVAL, SLIM_EDEVICE. */
slim_status slim_gram(slim_ctx* ctx, const int32_t* ids_a, int n_a, const int32_t* ids_b, int n_b,
                      double* out);

/* Checkpoint state: k, epoch, position in the epoch and the window's angle
 * ids.  The Gram is recomputed from the ids, so a restored run continues
 * bit-identically.  size in/out: bytes available / needed.
 * Errors: SLIM_EINVAL (buffer too small: *size is set), SLIM_ESTATE (bad blob). */
slim_status slim_get_state(slim_ctx* ctx, void* buf, int64_t* size);
slim_status slim_set_state(slim_ctx* ctx, const void* buf, int64_t size);

/* A group of contexts stepped together: grids of different sizes (e.g.
 * batches of 256^2, 512^2 and 1024^2 slices) scanned with the same angles and
 * block size.  slim_group_step applies one sampled block to every context:
 * the residual projections and explicit Gram solves of all contexts are
 * enqueued first, then the contexts' CG solves (in shared launches, see
 * slim_group_set_shared, or chunk by chunk under one host loop), then every
 * update.  The group
 * borrows the contexts, which must outlive it.
 * Errors: SLIM_EINVAL (NULL, n < 1, a context listed twice, contexts with
 * different n_angles or angles_per_block). */
typedef struct slim_group slim_group;
slim_status slim_group_create(slim_group** out, slim_ctx* const* ctxs, int n);

/* One step of every context of the group (eq. (ram) with the same block).
 *  infos  host [n] or NULL (then nothing is read back).
 * Errors: as slim_step, and SLIM_ESTATE for a context bound to streaming
 * data (b = NULL; step those with slim_step_data).  A step refused before any
 * device work (bad ids, no data, streaming data, a workspace that does not
 * fit) leaves every context as it was; after a device error every context
 * of the group is left unbound and must be rebound with slim_set_data. */
slim_status slim_group_step(slim_group* g, const int32_t* angle_ids, int n_ids,
                            slim_step_info* infos);

/* How the group's CG solves run: independent problems of different sizes
 * batched into shared launches, or not.  on = 1 (groups of at most 16
 * contexts): the solves of all contexts in CG mode
 * advance in the same launches -- per iteration one back-projection, one
 * forward projection (band kernel and reduction) and one vector kernel over
 * every context's slices, each workgroup finding its context in a table of
 * descriptors in device memory -- on the first such context's stream, with
 * chunks of iterations replayed as one graph; the other contexts' streams
 * hand over and take back their work by events.  Each slice still stops at
 * its own tolerance, and the results equal those of on = 0 (the default),
 * where each context's solve uses its own launches and one host loop
 * interleaves them; contexts on different streams then also overlap on the
 * GPU, which hides the kernel boundaries that shared launches keep (on the
 * 64 x 256^2 + 32 x 512^2 + 8 x 1024^2 batch shared launches take 32 ms per
 * step, interleaved ones 27 ms, one context after another 36 ms).  While
 * kernel timing (slim_profile) is on in a context, the group uses on = 0 for
 * that step.
 * Errors: SLIM_EINVAL (NULL group, on not 0 or 1, on = 1 with more than 16
 * contexts). */
slim_status slim_group_set_shared(slim_group* g, int on);
void slim_group_destroy(slim_group* g);

/* Launch shape of the projectors.  Zero fields take the built-in rules. */
typedef struct {
  int fwd_bt;       /* forward slice tile: 0, 1, 2 or 4                      */
  int fwd_items;    /* cap on forward rays per lane: 0, 2, 3, 4, 6, 8 or 10;
                       caps above the tile's maximum (8, 6, 3 rays for tiles
                       of 1, 2, 4 slices) act as that maximum               */
  int fwd_slots;    /* forward workgroups per CU the grid aims at: 0, 2 or 4 */
  int back_bt;      /* back-projector slice tile: 0, 1, 2 or 4               */
} slim_tune;

typedef struct {
  slim_tune chosen;         /* the fastest shape measured                    */
  double fwd_us, back_us;   /* its forward and back times on the window      */
  double fwd_default_us;    /* the built-in rules' times on the same window  */
  double back_default_us;
  int candidates;           /* shapes measured                               */
  int cached;               /* 1: taken from this process's earlier search    */
} slim_tune_info;

/* Autotuner: time every projector launch shape on forward and back
 * projections of a list of angles for all slices (three interleaved rounds
 * of a warm-up and three timed launches each; a shape scores its fastest
 * round), and keep the fastest (including the built-in rules) for lists of
 * that size.  n_ids = 0 tunes the
 * CG workload -- a window of (r+1) blocks of angles_per_block angles spread
 * over [0, pi) -- and also makes its shape the default for every other size;
 * n_ids > 0 (at most min(256, n_angles)) tunes a block of n_ids adjacent
 * angles (e.g. angles_per_block, for the residual and single-block
 * projections), scored by the sum of its times from angle 0 (row-stepping)
 * and from angle n_angles/2 (column-stepping) when 2 n_ids <= n_angles.  Results are cached per (N, n_slices, n_rays, list size) for
 * the process; force != 0 measures again.  Uses temporary device memory of
 * about 2 images and the list's rays per slice.  info may be NULL.
 * Errors: SLIM_EINVAL, SLIM_ENOMEM, SLIM_EDEVICE. */
slim_status slim_autotune(slim_ctx* ctx, int n_ids, int force, slim_tune_info* info);

/* Set (or read back, with get) the default projector launch shape; set also
 * drops the shapes tuned for particular list sizes.  Every shape computes the
 * same projections (to float32 rounding order).
 * Errors: SLIM_EINVAL (NULL, or a field outside its listed values). */
slim_status slim_set_tune(slim_ctx* ctx, const slim_tune* tune);
slim_status slim_get_tune(slim_ctx* ctx, slim_tune* tune);

/* Per-kernel timing (measurement support).  slim_profile(ctx, 1) resets the
 * counters and brackets every subsequent projector / Gram / Cholesky / CG
 * vector launch group with HIP events on the context's stream; 0 stops.
 * slim_kernel_stats returns the summed event time (ms) and the number of
 * timed launch groups of one kind: 0 forward projector's band kernel in CG
 * products (M u over the window), 1 back-projector in CG products (M^T v over
 * the window), 2 Gram blocks and assembly, 3 Cholesky factorisation and
 * solves, 4 CG vector kernels, 5 residual forward projection of the new
 * block, 6 fused back-projection and update of x, 7 the reduction of the CG
 * forward products.  Both synchronise the stream.
 * Errors: SLIM_EINVAL (NULL arguments, unknown kind), SLIM_EDEVICE. */
slim_status slim_profile(slim_ctx* ctx, int on);
slim_status slim_kernel_stats(slim_ctx* ctx, int kind, double* total_ms, int64_t* launches);

/* Release every device allocation of ctx (NULL is a no-op). */
void slim_destroy(slim_ctx* ctx);

/* Static description of a status code. */
const char* slim_strerror(slim_status s);

/* Message of the last failing call on this thread ("" if none). */
const char* slim_last_error(void);

#ifdef __cplusplus
}
#endif

#endif /* SLIM_H */
