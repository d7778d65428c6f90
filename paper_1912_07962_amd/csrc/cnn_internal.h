// Launchers of the warm-start CNN kernels (cnn.hip).  Tensors are NHWC:
// [batch][row][column][channel stride], channels of one tensor may live in a
// slice [co, co + C) of a wider buffer (the U-Net's concatenations), bf16
// stored as uint16_t.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "../../include/slim_cnn.h"

namespace slim {
namespace cnn {

struct Tensor {
  uint16_t* p = nullptr;   // bf16 [B][H][H][cs]
  int cs = 0;              // channel stride
  int co = 0;              // first channel
};

// out = act(conv3x3(in) + bias), optionally times (mask > 0).  The conv runs
// on the H x H output grid; with up != 0 the input is H/2 x H/2 and is read
// nearest-upsampled.  w: bf16 [Cout][3][3][Cin].  Requires Cin, Cout
// multiples of 32, H*H a multiple of 64, channel offsets/strides multiples
// of 8.
struct ConvArgs {
  Tensor in;
  int Cin = 0, up = 0;
  const uint16_t* w = nullptr;
  const float* bias = nullptr;
  Tensor out;
  int Cout = 0;
  Tensor mask;   // mask.p == nullptr: no mask
  int relu = 0;
  int B = 0, H = 0;
};
hipError_t launch_conv3x3(const ConvArgs& a, hipStream_t st);

// Weight and bias gradients of a conv3x3: dW[co][tap][ci] = sum_p dz[p][co]
// x_tap[p][ci], db[co] = sum_p dz[p][co], as fixed-order split-K partials
// reduced into dw (fp32 [Cout][9][Cin]) and db (fp32 [Cout]).  part is a
// workspace of wgrad_part_floats() floats.
struct WgradArgs {
  Tensor dz;
  int Cout = 0;
  Tensor in;
  int Cin = 0, up = 0;
  int B = 0, H = 0;
  float* dw = nullptr;
  float* db = nullptr;
  float* part = nullptr;
};
size_t wgrad_part_floats(int Cout, int Cin, int B, int H);
hipError_t launch_wgrad(const WgradArgs& a, hipStream_t st);

// First layer (one input channel, fp32 input scaled by in_scale):
// out = relu(conv3x3(in_scale * u) + bias), w bf16 [Cout][3][3][1].
hipError_t launch_conv_in(const float* u, double in_scale, const uint16_t* w, const float* bias,
                          Tensor out, int Cout, int B, int H, hipStream_t st);
size_t wgrad_in_part_floats(int Cout, int B, int H);
hipError_t launch_wgrad_in(const uint16_t* dz, int Cout, const float* u, double in_scale, int B,
                           int H, float* dw, float* db, float* part, hipStream_t st);

// 2x2 average pool: out (H/2 grid, C channels) from in (H grid).
hipError_t launch_pool(Tensor in, Tensor out, int C, int B, int H, hipStream_t st);
// dE[q] = (dE[q] + dp[parent(q)] / 4) * (E[q] > 0) in place (H grid).
hipError_t launch_pool_back_add(Tensor dp, Tensor e, Tensor de, int C, int B, int H,
                                hipStream_t st);
// dD[q] = (sum of du over the 4 children of q) * (D[q] > 0); q on the H grid,
// du on the 2H grid.
hipError_t launch_up_back(Tensor du, Tensor d, Tensor dd, int C, int B, int H, hipStream_t st);

// x0[p] = sum_c wh[c] D[p][c] + bh + cu * in_scale * u[p]; head = {wh[C], bh, cu}.
hipError_t launch_head(Tensor d, int C, const float* head, const float* u, double in_scale,
                       float* x0, int64_t npx, hipStream_t st);
// Loss and head backward: diff = x0 - t; dz[p][c] = bf16(2 diff/npx wh[c]
// (D > 0)); partials of (sum diff^2, d wh[c], d bh, d cu) per workgroup,
// reduced in fixed order into loss (fp64) and dhead (fp32 [C+2]).
size_t head_part_doubles(int C, int64_t npx);
hipError_t launch_head_back(Tensor d, int C, const float* head, const float* u, double in_scale,
                            const float* x0, const float* target, int64_t npx, Tensor dz,
                            double* part, double* loss, float* dhead, hipStream_t st);

// Adam over n fp32 entries with bias-corrected step sizes precomputed on the
// host: p -= lr_t * m / (sqrt(v) + eps_t).
hipError_t launch_adam(float* p, const float* g, float* m, float* v, int64_t n, float beta1,
                       float beta2, float lr_t, float eps_t, hipStream_t st);
// bf16 copies of a conv layer's weights: w16 [Cout][9][Cin] and the
// flipped transpose wt16 [Cin][9][Cout] (wt16[ci][8-t][co] = w[co][t][ci]),
// used by the data gradient.
hipError_t launch_cast_weights(const float* w, uint16_t* w16, uint16_t* wt16, int Cout, int Cin,
                               hipStream_t st);
// x = 0 for n floats.
hipError_t launch_zero(float* x, int64_t n, hipStream_t st);

}  // namespace cnn
}  // namespace slim

// Used by the warm start of a slimLS context (slim_api.cpp).
slim_status cnn_forward_on(slim_cnn* net, const float* u, float* x0, int B, hipStream_t st);
bool cnn_usable(const slim_cnn* net);
int cnn_side(const slim_cnn* net);
int cnn_max_batch(const slim_cnn* net);
