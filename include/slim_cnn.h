/* Learned warm start for slimLS: a small U-Net maps the back-projection of
 * the first sampled blocks, u = sum_j A_{tau_j}^T b_{tau_j}, to a starting
 * point x0 (the iteration of eq. (ram) starts from any x0; its updates lie in
 * R(A^T), sec. 1).
 *
 * Network (levels L in 2..4, channels c_1..c_L, image N x N, one channel):
 *   uh = in_scale * u
 *   E_1 = relu(conv(relu(conv(uh))))                  c_1 channels, N x N
 *   E_l = relu(conv(relu(conv(pool(E_{l-1})))))       c_l channels, N/2^(l-1)
 *   D_L = E_L;  for l = L-1 .. 1:
 *     U_l = relu(conv(up(D_{l+1})));  C_l = [U_l, E_l]   (channel concatenation)
 *     D_l = relu(conv(relu(conv(C_l))))                c_l channels
 *   x0 = sum_c wh[c] D_1[c] + bh + cu * uh
 * conv: 3x3 cross-correlation, zero padding, bias; pool: 2x2 average;
 * up: nearest x2.  Convolutions run on bf16 operands with fp32 accumulation;
 * activations and activation gradients are stored in bf16; parameters,
 * weight gradients and the Adam state are fp32.
 *
 * Parameters are one packed fp32 vector, layer by layer in forward order
 * (e1a e1b e2a e2b ... eLa eLb, then for l = L-1..1: u_l d_la d_lb), each
 * layer as weights [Cout][3][3][Cin] followed by bias [Cout]; then wh [c_1],
 * bh, cu.  Loss: mean squared error over images and pixels; optimizer: Adam
 * (Kingma & Ba 2015) with bias correction.
 *
 * All tensors passed in are device memory owned by the caller; images are
 * [batch][N][N] float32.  A network is bound to one device and stream and is
 * not thread-safe.  Status codes are those of slim.h. */
#ifndef SLIM_CNN_H
#define SLIM_CNN_H

#include "slim.h"

#ifdef __cplusplus
extern "C" {
#endif

typedef struct slim_cnn slim_cnn;

typedef struct {
  int N;             /* image side; a multiple of 8 * 2^(levels-1)           */
  int levels;        /* 2..4                                                 */
  int channels[4];   /* c_1..c_levels, multiples of 32, at most 512          */
  int max_batch;     /* images per call, >= 1                                */
  double in_scale;   /* uh = in_scale * u, finite and > 0                    */
  void* stream;      /* hipStream_t work queue (NULL = the default stream)    */
} slim_cnn_desc;

/* Create a network with zero parameters (set them with slim_cnn_set_params).
 * Errors: SLIM_EINVAL (desc out of range), SLIM_ENOMEM, SLIM_EDEVICE. */
slim_status slim_cnn_create(slim_cnn** out, const slim_cnn_desc* desc);

/* Number of fp32 entries of the packed parameter vector (0 for NULL). */
int64_t slim_cnn_num_params(const slim_cnn* net);

/* Copy the packed parameters in from / out to host memory (n entries).
 * set_params marks the network invalid if any entry is not finite (the warm
 * start then falls back to x0 = 0) and resets the Adam state.
 * Errors: SLIM_EINVAL (NULL or n != slim_cnn_num_params). */
slim_status slim_cnn_set_params(slim_cnn* net, const float* host, int64_t n);
slim_status slim_cnn_get_params(slim_cnn* net, float* host, int64_t n);

/* x0 = net(u) for B images: u, x0 device [B][N][N] float32, 1 <= B <= max_batch.
 * Errors: SLIM_EINVAL, SLIM_ESTATE (invalid parameters), SLIM_EDEVICE. */
slim_status slim_cnn_forward(slim_cnn* net, const float* u, float* x0, int B);

/* Forward and backward pass of the loss mean((net(u) - target)^2) over B
 * images; the gradient stays in the network (packed like the parameters).
 * loss (host, may be NULL) receives the loss; grad_host (may be NULL)
 * receives a copy of the gradient (slim_cnn_num_params entries).
 * Errors: as slim_cnn_forward. */
slim_status slim_cnn_loss_grad(slim_cnn* net, const float* u, const float* target, int B,
                               double* loss, float* grad_host);

/* One Adam step with the gradient of the last slim_cnn_loss_grad; the step
 * counter starts at 1 after create / set_params.
 * Errors: SLIM_EINVAL (lr <= 0, betas outside [0, 1), eps <= 0),
 * SLIM_ESTATE (no gradient yet), SLIM_EDEVICE. */
slim_status slim_cnn_adam(slim_cnn* net, double lr, double beta1, double beta2, double eps);

/* Warm start for the data bound to ctx (slim_set_data): u = A_ids^T b for the
 * listed angles (host int32, the angles of the first sampled blocks), then
 * x0 = net(u) for every slice, in chunks of max_batch.  With net == NULL or
 * invalid parameters x0 = 0 and *used_net = 0 (the fallback); otherwise
 * *used_net = 1.  x0: device [n_slices][N][N] float32.  If x0 is the image
 * bound by slim_set_data, the iteration restarts from it (k = 0, empty
 * memory window, as after slim_set_data).  Uses ctx's stream.
 * Errors: SLIM_EINVAL (bad ids, NULL x0, net->N != N), SLIM_ESTATE (no data
 * bound), SLIM_EDEVICE. */
slim_status slim_warmstart(slim_ctx* ctx, slim_cnn* net, const int32_t* angle_ids, int n_ids,
                           float* x0, int* used_net);

/* The network's FLOP count of one forward pass per image (2 per multiply-add
 * of the convolutions), for throughput reports. */
double slim_cnn_forward_flops(const slim_cnn* net);

void slim_cnn_destroy(slim_cnn* net);

#ifdef __cplusplus
}
#endif

#endif /* SLIM_CNN_H */
