/*
 * slim3d.h -- C ABI of the 3D parallel-beam slimLS path (MI355X, gfx950).
 *
 * The paper's 3D experiment (sec. 4.3, three-dimensional streaming
 * tomography) reconstructs a volume from projection images taken from
 * directions drawn uniformly on the unit sphere; one image is one block of
 * rows A_k, and slimLS (sec. 1, eq. (ram), eq. (B_k), C_k = I,
 * alpha_k = 1/lambda) iterates
 *
 *     x_k = x_{k-1} - (lambda I + M_k^T M_k)^{-1} A_k^T (A_k x_{k-1} - b_k),
 *     M_k = [A_{k-r}; ...; A_k],
 *
 * computed here in the Gram form s = M^T z, (M M^T + lambda I) z =
 * [0; ...; 0; A_k x - b_k], the Gram system solved by conjugate gradients
 * with matrix-free projectors (a block has n_det^2 rows, so the Gram matrix
 * is never formed), by default preconditioned by the inverse of the Gram
 * diagonal: a ray's squared weights vary with its chord through the cube,
 * and scaling them out cuts the iterations several-fold for one image.
 *
 * Geometry: the volume covers [-1, 1]^3 with N^3 voxels of side h = 2/N,
 * stored [k][i][j] = (z, y, x) row-major, voxel centre ((j, i, k) - (N-1)/2) h.
 * A direction w (unit vector) has the detector basis e_u = (z x w)/|z x w|
 * (e_u = x when w = +-z) and e_v = w x e_u; its image has n_det x n_det
 * pixels of side h, pixel (q, t) on the ray {u_t e_u + v_q e_v + tau w},
 * u_t = (t - (n_det-1)/2) h, v_q likewise, stored [q][t].  Weights are
 * Joseph's method along the major axis m of w (largest |w_m|, the first on a
 * tie): the ray crosses each plane x_m = const through voxel centres once,
 * and in that plane it takes the bilinear interpolation of the four voxel
 * centres around the crossing point, times h / |w_m|:
 *     a(ray, voxel) = (h/|w_m|) max(0, 1 - |P_a - c_a|/h) max(0, 1 - |P_b - c_b|/h),
 * P the crossing point in the voxel's plane, a and b the other two axes.
 * Voxels outside the volume are zero.
 *
 * Conventions as in slim.h: device arrays are caller-owned and borrowed for
 * the call (b, x and x_true until the next slim3d_set_data); work runs on
 * opts.stream; calls that return host-visible numbers synchronise it; every
 * error is a slim_status, checked before any device work.  A context is
 * bound to one device and one stream and is not thread-safe.
 */
#ifndef SLIM3D_H
#define SLIM3D_H

#include <stdint.h>

#include "slim.h"

#ifdef __cplusplus
extern "C" {
#endif

typedef struct slim3d_ctx slim3d_ctx;

/* Create a context.
 *  N         voxels per side, 2 <= N <= 1024
 *  n_dirs    number of projection directions (>= 1)
 *  dirs      host float64 [n_dirs][3], each of unit length (|1 - |w|| <= 1e-6)
 *  n_det     detector pixels per side, 1 <= n_det <= 4096
 *  r         memory level r >= 0 (the paper's 3D run uses r = 0)
 *  lambda    damping 1/alpha > 0, finite
 *  opts      host or NULL; used fields: angles_per_block (directions per
 *            block, g, must divide n_dirs; (r+1) g <= 256), pcg_tol,
 *            pcg_max_iter, gram_mode, stream.  gram_mode AUTO or JACOBI:
 *            CG preconditioned by the inverse Gram diagonal; PCG: plain CG
 *            (either way the stop test is ||res|| <= pcg_tol ||rhs|| on
 *            the Gram system's residual, not the preconditioned one); CHOL
 *            is refused.  Other fields must hold
 *            their defaults' meaning for this path: precision FP32,
 *            tikhonov 0.
 * Allocates the direction table and the step workspace: three padded
 * volumes of N^2 (N + 11) floats at most (the volume stored with x, y or z
 * slowest, rows on 16-byte boundaries, which the forward projector reads
 * for directions of that major axis: copies of x and the CG's M^T p), five
 * float64 vectors of (r+1) g n_det^2 entries (right-hand side, residual,
 * direction, product, solution) and one more with JACOBI (the
 * preconditioner), the forward projector's per-segment ray sums (eight
 * float64 values per ray of (r+1) g images) and small reduction buffers.
 * Errors: SLIM_EINVAL, SLIM_ENOMEM, SLIM_EDEVICE. */
slim_status slim3d_init(slim3d_ctx** out, int N, int n_dirs, const double* dirs, int n_det, int r,
                        double lambda, const slim_opts* opts);

/* Bind the data (sec. 1, eq. (inverseproblem)).
 *  b       device float32 [n_dirs][n_det][n_det], the projection images
 *  x       device float32 [N][N][N], the iterate (read and overwritten)
 *  x_true  device float32 [N][N][N] or NULL (enables err_norm)
 * Resets the iteration (k = 0, empty memory window).
 * Errors: SLIM_EINVAL on NULL b or x. */
slim_status slim3d_set_data(slim3d_ctx* ctx, const float* b, float* x, const float* x_true);

/* One slimLS iteration (eq. (ram)) with the block of the given directions
 * (host int32 [n_ids], n_ids == angles_per_block, each in [0, n_dirs), no
 * duplicates): residual of the block, CG on the window's Gram system (to
 * ||res|| <= pcg_tol ||rhs||, at most pcg_max_iter iterations, float64
 * scalars and vectors), back-projection over the window and update of x,
 * float64 norms.  info may be NULL (then nothing is read back; the CG's
 * host loop still synchronises the stream between chunks of iterations).
 * Errors: SLIM_EINVAL (bad ids), SLIM_ESTATE (no data), SLIM_ENUMERIC
 * (non-finite data, iterate or norm), SLIM_ENOTCONV (CG cap reached; the
 * step is applied), SLIM_EDEVICE (the context is left unbound: rebind with
 * slim3d_set_data). */
slim_status slim3d_step(slim3d_ctx* ctx, const int32_t* dir_ids, int n_ids, slim_step_info* info);

/* Forward projection out = A_ids x (ids host int32 [n_ids], repeats allowed,
 * n_ids <= 256): x device float32 [N][N][N], out device float32
 * [n_ids][n_det][n_det].  Ray sums accumulate in float64.
 * Errors: SLIM_EINVAL, SLIM_EDEVICE. */
slim_status slim3d_project(slim3d_ctx* ctx, const int32_t* dir_ids, int n_ids, const float* x,
                           float* out);

/* Back-projection out = A_ids^T v, the exact adjoint of slim3d_project:
 * v device float32 [n_ids][n_det][n_det], out device float32 [N][N][N]
 * (overwritten).  Errors: SLIM_EINVAL, SLIM_EDEVICE. */
slim_status slim3d_backproject(slim3d_ctx* ctx, const int32_t* dir_ids, int n_ids,
                               const float* v, float* out);

/* Per-kernel timing, as slim_profile / slim_kernel_stats: kinds 0 forward
 * projector in CG products, 1 back-projector in CG products, 4 CG vector
 * kernels, 5 residual forward projection, 6 back-projection and update. */
slim_status slim3d_profile(slim3d_ctx* ctx, int on);
slim_status slim3d_kernel_stats(slim3d_ctx* ctx, int kind, double* total_ms, int64_t* launches);

/* Release every device allocation of ctx (NULL is a no-op). */
void slim3d_destroy(slim3d_ctx* ctx);

#ifdef __cplusplus
}
#endif

#endif /* SLIM3D_H */
