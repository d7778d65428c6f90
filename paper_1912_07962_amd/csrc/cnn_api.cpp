// C ABI of the warm-start CNN: parameters, activation buffers, the forward
// and backward schedules of the U-Net, Adam, and the warm start itself.
//
// Buffers (bf16, NHWC, level l = 0..L-1 at resolution H_l = N >> l with
// c_l channels):
//   A[l]    output of e(l+1)a
//   Cat[l]  l < L-1: [U_l | E_l] (2 c_l channels); E_l is written straight
//           into its second half by e(l+1)b, U_l into its first half
//   EL      E_{L-1} (the bottom level has no concatenation)
//   P[l]    pool(E_l), l < L-1, at resolution H_{l+1}
//   Da[l], D[l]   outputs of d(l+1)a, d(l+1)b, l < L-1
//   dCat[l] gradient at Cat[l]'s pre-activations, kept from the decoder
//           pass to the encoder pass (its second half receives the pool path)
//   G1..G3  gradient scratch
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstring>
#include <string>
#include <vector>

#include "../../include/slim_cnn.h"
#include "cnn_internal.h"
#include "slim_internal.h"

using namespace slim;
using slim::cnn::Tensor;

namespace {

#define CNN_TRY(expr)                                                                    \
  do {                                                                                   \
    hipError_t _e = (expr);                                                              \
    if (_e != hipSuccess)                                                                \
      return set_error(SLIM_EDEVICE, std::string(#expr) + ": " + hipGetErrorString(_e)); \
  } while (0)

struct Layer {
  int Cout = 0, Cin = 0;
  int64_t off_w = 0, off_b = 0;  // in the packed fp32 vectors
  int64_t off16 = 0;             // in the bf16 weight copies
};

template <typename T>
hipError_t dalloc(T** p, size_t count) {
  *p = nullptr;
  if (count == 0) return hipSuccess;
  return hipMalloc((void**)p, count * sizeof(T));
}

}  // namespace

struct slim_cnn {
  int N = 0, L = 0, maxB = 0;
  int c[4] = {0, 0, 0, 0};
  double in_scale = 1.0;
  hipStream_t st = nullptr;
  std::vector<Layer> layers;   // e1a e1b ... eLa eLb, then u_l d_la d_lb for l = L-1..1
  int64_t n_params = 0, off_head = 0, n16 = 0;
  float *p = nullptr, *g = nullptr, *m = nullptr, *v = nullptr;
  uint16_t *w16 = nullptr, *wt16 = nullptr;
  bool valid = false, have_grad = false;
  int t = 0;
  std::vector<uint16_t*> A, Cat, P, Da, D, dCat;
  uint16_t* EL = nullptr;
  uint16_t *G1 = nullptr, *G2 = nullptr, *G3 = nullptr;
  float* x0buf = nullptr;
  float* wpart = nullptr;
  double* hpart = nullptr;
  double* d_loss = nullptr;
  double* h_loss = nullptr;

  int H(int l) const { return N >> l; }
  int e_a(int l) const { return 2 * l; }       // layer index of e(l+1)a
  int e_b(int l) const { return 2 * l + 1; }
  int u_(int l) const { return 2 * L + 3 * (L - 2 - l); }   // u(l+1), l = L-2..0
  int d_a(int l) const { return u_(l) + 1; }
  int d_b(int l) const { return u_(l) + 2; }
  Tensor E(int l) const {
    if (l == L - 1) return Tensor{EL, c[l], 0};
    return Tensor{Cat[l], 2 * c[l], c[l]};
  }

  ~slim_cnn() {
    for (void* q : {(void*)p, (void*)g, (void*)m, (void*)v, (void*)w16, (void*)wt16, (void*)EL,
                    (void*)G1, (void*)G2, (void*)G3, (void*)x0buf, (void*)wpart, (void*)hpart,
                    (void*)d_loss})
      (void)hipFree(q);
    for (auto* vec : {&A, &Cat, &P, &Da, &D, &dCat})
      for (uint16_t* q : *vec) (void)hipFree(q);
    if (h_loss) (void)hipHostFree(h_loss);
  }
};

namespace {

slim_status cnn_fail(slim_status s, const std::string& msg) { return set_error(s, msg); }

hipError_t cast_all(slim_cnn* n) {
  for (const Layer& ly : n->layers) {
    hipError_t e = cnn::launch_cast_weights(n->p + ly.off_w, n->w16 + ly.off16,
                                            ly.Cin == 1 ? nullptr : n->wt16 + ly.off16, ly.Cout,
                                            ly.Cin, n->st);
    if (e != hipSuccess) return e;
  }
  return hipSuccess;
}

// conv through the MFMA kernel with the layer's forward weights
hipError_t conv_fwd(slim_cnn* n, int li, Tensor in, int up, Tensor out, int B, int H) {
  const Layer& ly = n->layers[li];
  cnn::ConvArgs a;
  a.in = in;
  a.Cin = ly.Cin;
  a.up = up;
  a.w = n->w16 + ly.off16;
  a.bias = n->p + ly.off_b;
  a.out = out;
  a.Cout = ly.Cout;
  a.relu = 1;
  a.B = B;
  a.H = H;
  return cnn::launch_conv3x3(a, n->st);
}

// gradient at the layer's input from dz (gradient at its pre-activation),
// optionally masked by (mask > 0); H is the layer's output grid
hipError_t conv_bwd(slim_cnn* n, int li, Tensor dz, Tensor mask, Tensor out, int B, int H) {
  const Layer& ly = n->layers[li];
  cnn::ConvArgs a;
  a.in = dz;
  a.Cin = ly.Cout;
  a.up = 0;
  a.w = n->wt16 + ly.off16;
  a.bias = nullptr;
  a.out = out;
  a.Cout = ly.Cin;
  a.mask = mask;
  a.relu = 0;
  a.B = B;
  a.H = H;
  return cnn::launch_conv3x3(a, n->st);
}

hipError_t wgrad(slim_cnn* n, int li, Tensor dz, Tensor in, int up, int B, int H) {
  const Layer& ly = n->layers[li];
  cnn::WgradArgs a;
  a.dz = dz;
  a.Cout = ly.Cout;
  a.in = in;
  a.Cin = ly.Cin;
  a.up = up;
  a.B = B;
  a.H = H;
  a.dw = n->g + ly.off_w;
  a.db = n->g + ly.off_b;
  a.part = n->wpart;
  return cnn::launch_wgrad(a, n->st);
}

hipError_t forward(slim_cnn* n, const float* u, float* x0, int B) {
  hipError_t e;
  const int L = n->L;
  const Layer& l0 = n->layers[n->e_a(0)];
  if ((e = cnn::launch_conv_in(u, n->in_scale, n->w16 + l0.off16, n->p + l0.off_b,
                               Tensor{n->A[0], n->c[0], 0}, n->c[0], B, n->N, n->st)) != hipSuccess)
    return e;
  if ((e = conv_fwd(n, n->e_b(0), Tensor{n->A[0], n->c[0], 0}, 0, n->E(0), B, n->H(0))) != hipSuccess)
    return e;
  for (int l = 1; l < L; ++l) {
    const Tensor pl{n->P[l - 1], n->c[l - 1], 0};
    if ((e = cnn::launch_pool(n->E(l - 1), pl, n->c[l - 1], B, n->H(l - 1), n->st)) != hipSuccess)
      return e;
    if ((e = conv_fwd(n, n->e_a(l), pl, 0, Tensor{n->A[l], n->c[l], 0}, B, n->H(l))) != hipSuccess)
      return e;
    if ((e = conv_fwd(n, n->e_b(l), Tensor{n->A[l], n->c[l], 0}, 0, n->E(l), B, n->H(l))) !=
        hipSuccess)
      return e;
  }
  Tensor below = n->E(L - 1);
  for (int l = L - 2; l >= 0; --l) {
    const Tensor cat{n->Cat[l], 2 * n->c[l], 0};
    if ((e = conv_fwd(n, n->u_(l), below, 1, cat, B, n->H(l))) != hipSuccess) return e;
    if ((e = conv_fwd(n, n->d_a(l), cat, 0, Tensor{n->Da[l], n->c[l], 0}, B, n->H(l))) != hipSuccess)
      return e;
    if ((e = conv_fwd(n, n->d_b(l), Tensor{n->Da[l], n->c[l], 0}, 0, Tensor{n->D[l], n->c[l], 0},
                      B, n->H(l))) != hipSuccess)
      return e;
    below = Tensor{n->D[l], n->c[l], 0};
  }
  return cnn::launch_head(Tensor{n->D[0], n->c[0], 0}, n->c[0], n->p + n->off_head, u,
                          n->in_scale, x0, (int64_t)B * n->N * n->N, n->st);
}

hipError_t backward(slim_cnn* n, const float* u, const float* target, int B) {
  hipError_t e;
  const int L = n->L;
  const int64_t npx = (int64_t)B * n->N * n->N;
  const Tensor none{};
  if ((e = cnn::launch_head_back(Tensor{n->D[0], n->c[0], 0}, n->c[0], n->p + n->off_head, u,
                                 n->in_scale, n->x0buf, target, npx, Tensor{n->G1, n->c[0], 0},
                                 n->hpart, n->d_loss, n->g + n->off_head, n->st)) != hipSuccess)
    return e;
  Tensor dy{n->G1, n->c[0], 0};
  // decoder, top level first
  for (int l = 0; l <= L - 2; ++l) {
    const int H = n->H(l), cl = n->c[l], cb = n->c[l + 1];
    const Tensor da{n->Da[l], cl, 0}, cat{n->Cat[l], 2 * cl, 0}, dcat{n->dCat[l], 2 * cl, 0};
    const Tensor g2{n->G2, cl, 0};
    if ((e = conv_bwd(n, n->d_b(l), dy, da, g2, B, H)) != hipSuccess) return e;
    if ((e = wgrad(n, n->d_b(l), dy, da, 0, B, H)) != hipSuccess) return e;
    if ((e = conv_bwd(n, n->d_a(l), g2, cat, dcat, B, H)) != hipSuccess) return e;
    if ((e = wgrad(n, n->d_a(l), g2, cat, 0, B, H)) != hipSuccess) return e;
    const Tensor below = l + 1 < L - 1 ? Tensor{n->D[l + 1], cb, 0} : n->E(L - 1);
    const Tensor g3{n->G3, cb, 0};
    if ((e = conv_bwd(n, n->u_(l), dcat, none, g3, B, H)) != hipSuccess) return e;
    if ((e = wgrad(n, n->u_(l), dcat, below, 1, B, H)) != hipSuccess) return e;
    const Tensor g1{n->G1, cb, 0};
    if ((e = cnn::launch_up_back(g3, below, g1, cb, B, n->H(l + 1), n->st)) != hipSuccess) return e;
    dy = g1;
  }
  // encoder, bottom level first
  for (int l = L - 1; l >= 0; --l) {
    const int H = n->H(l), cl = n->c[l];
    const Tensor dye = l == L - 1 ? dy : Tensor{n->dCat[l], 2 * cl, cl};
    const Tensor a{n->A[l], cl, 0}, g2{n->G2, cl, 0};
    if ((e = conv_bwd(n, n->e_b(l), dye, a, g2, B, H)) != hipSuccess) return e;
    if ((e = wgrad(n, n->e_b(l), dye, a, 0, B, H)) != hipSuccess) return e;
    if (l == 0) {
      const Layer& ly = n->layers[n->e_a(0)];
      if ((e = cnn::launch_wgrad_in(n->G2, cl, u, n->in_scale, B, H, n->g + ly.off_w,
                                    n->g + ly.off_b, n->wpart, n->st)) != hipSuccess)
        return e;
      break;
    }
    const int cp = n->c[l - 1];
    const Tensor g3{n->G3, cp, 0};
    if ((e = conv_bwd(n, n->e_a(l), g2, none, g3, B, H)) != hipSuccess) return e;
    if ((e = wgrad(n, n->e_a(l), g2, Tensor{n->P[l - 1], cp, 0}, 0, B, H)) != hipSuccess) return e;
    if ((e = cnn::launch_pool_back_add(g3, n->E(l - 1), Tensor{n->dCat[l - 1], 2 * cp, cp}, cp, B,
                                       n->H(l - 1), n->st)) != hipSuccess)
      return e;
  }
  return hipSuccess;
}

slim_status check_batch(const slim_cnn* n, int B) {
  if (B < 1 || B > n->maxB)
    return cnn_fail(SLIM_EINVAL, "batch must be in [1, max_batch]");
  return SLIM_OK;
}

}  // namespace

slim_status cnn_forward_on(slim_cnn* n, const float* u, float* x0, int B, hipStream_t st) {
  hipStream_t keep = n->st;
  n->st = st;
  hipError_t e = forward(n, u, x0, B);
  n->st = keep;
  if (e != hipSuccess) return cnn_fail(SLIM_EDEVICE, std::string("cnn forward: ") + hipGetErrorString(e));
  return SLIM_OK;
}

bool cnn_usable(const slim_cnn* n) { return n && n->valid; }
int cnn_side(const slim_cnn* n) { return n->N; }
int cnn_max_batch(const slim_cnn* n) { return n->maxB; }

extern "C" {

slim_status slim_cnn_create(slim_cnn** out, const slim_cnn_desc* d) {
  if (!out || !d) return cnn_fail(SLIM_EINVAL, "out or desc is NULL");
  *out = nullptr;
  if (d->levels < 2 || d->levels > 4) return cnn_fail(SLIM_EINVAL, "levels must be in 2..4");
  for (int l = 0; l < d->levels; ++l)
    if (d->channels[l] < 32 || d->channels[l] > 512 || d->channels[l] % 32 != 0)
      return cnn_fail(SLIM_EINVAL, "channels must be multiples of 32 in [32, 512]");
  const int mult = 8 << (d->levels - 1);
  if (d->N < mult || d->N % mult != 0 || d->N > 8192)
    return cnn_fail(SLIM_EINVAL, "N must be a multiple of 8 * 2^(levels-1), at most 8192");
  if (d->max_batch < 1) return cnn_fail(SLIM_EINVAL, "max_batch must be >= 1");
  if (!std::isfinite(d->in_scale) || d->in_scale <= 0.0)
    return cnn_fail(SLIM_EINVAL, "in_scale must be finite and > 0");

  slim_cnn* n = new slim_cnn;
  n->N = d->N;
  n->L = d->levels;
  n->maxB = d->max_batch;
  n->in_scale = d->in_scale;
  n->st = (hipStream_t)d->stream;
  for (int l = 0; l < n->L; ++l) n->c[l] = d->channels[l];
  const int L = n->L;
  std::vector<std::pair<int, int>> shapes;   // (Cout, Cin) in layer order
  shapes.push_back({n->c[0], 1});
  shapes.push_back({n->c[0], n->c[0]});
  for (int l = 1; l < L; ++l) {
    shapes.push_back({n->c[l], n->c[l - 1]});
    shapes.push_back({n->c[l], n->c[l]});
  }
  for (int l = L - 2; l >= 0; --l) {
    shapes.push_back({n->c[l], n->c[l + 1]});
    shapes.push_back({n->c[l], 2 * n->c[l]});
    shapes.push_back({n->c[l], n->c[l]});
  }
  int64_t off = 0, off16 = 0;
  for (auto [co, ci] : shapes) {
    Layer ly;
    ly.Cout = co;
    ly.Cin = ci;
    ly.off_w = off;
    off += (int64_t)co * 9 * ci;
    ly.off_b = off;
    off += co;
    ly.off16 = off16;
    off16 += (int64_t)co * 9 * ci;
    n->layers.push_back(ly);
  }
  n->off_head = off;
  n->n_params = off + n->c[0] + 2;
  n->n16 = off16;

  auto oom = [&](hipError_t e) -> slim_status {
    delete n;
    if (e == hipErrorOutOfMemory || e == hipErrorMemoryAllocation)
      return cnn_fail(SLIM_ENOMEM, "device workspace does not fit");
    return cnn_fail(SLIM_EDEVICE, std::string("allocation: ") + hipGetErrorString(e));
  };
  hipError_t e;
  const size_t B = (size_t)n->maxB;
  if ((e = dalloc(&n->p, n->n_params)) != hipSuccess) return oom(e);
  if ((e = dalloc(&n->g, n->n_params)) != hipSuccess) return oom(e);
  if ((e = dalloc(&n->m, n->n_params)) != hipSuccess) return oom(e);
  if ((e = dalloc(&n->v, n->n_params)) != hipSuccess) return oom(e);
  if ((e = dalloc(&n->w16, n->n16)) != hipSuccess) return oom(e);
  if ((e = dalloc(&n->wt16, n->n16)) != hipSuccess) return oom(e);
  size_t g1 = 0, g2 = 0, g3 = 0, wp = 0;
  for (int l = 0; l < L; ++l) {
    const size_t px = B * n->H(l) * n->H(l);
    uint16_t* q = nullptr;
    if ((e = dalloc(&q, px * n->c[l])) != hipSuccess) return oom(e);
    n->A.push_back(q);
    g2 = std::max(g2, px * n->c[l]);
    if (l < L - 1) {
      const size_t pxn = B * n->H(l + 1) * n->H(l + 1);
      for (auto* vec : {&n->Cat, &n->dCat}) {
        if ((e = dalloc(&q, px * 2 * n->c[l])) != hipSuccess) return oom(e);
        vec->push_back(q);
      }
      if ((e = dalloc(&q, pxn * n->c[l])) != hipSuccess) return oom(e);
      n->P.push_back(q);
      for (auto* vec : {&n->Da, &n->D}) {
        if ((e = dalloc(&q, px * n->c[l])) != hipSuccess) return oom(e);
        vec->push_back(q);
      }
      g1 = std::max(g1, px * n->c[l]);                    // head / up_back at level l
      g1 = std::max(g1, pxn * n->c[l + 1]);
      g3 = std::max(g3, px * n->c[l + 1]);                // gradient at up(D_{l+1})
    } else {
      if ((e = dalloc(&n->EL, px * n->c[l])) != hipSuccess) return oom(e);
    }
    if (l > 0) g3 = std::max(g3, px * n->c[l - 1]);      // gradient at pool(E_{l-1})
  }
  for (const Layer& ly : n->layers) {
    const int li = (int)(&ly - n->layers.data());
    int H = n->N;
    for (int l = 0; l < L; ++l)
      if (li == n->e_a(l) || li == n->e_b(l) || (l < L - 1 && (li == n->u_(l) || li == n->d_a(l) ||
                                                                li == n->d_b(l))))
        H = n->H(l);
    wp = std::max(wp, ly.Cin == 1 ? cnn::wgrad_in_part_floats(ly.Cout, (int)B, H)
                                  : cnn::wgrad_part_floats(ly.Cout, ly.Cin, (int)B, H));
  }
  if ((e = dalloc(&n->G1, g1)) != hipSuccess) return oom(e);
  if ((e = dalloc(&n->G2, g2)) != hipSuccess) return oom(e);
  if ((e = dalloc(&n->G3, g3)) != hipSuccess) return oom(e);
  if ((e = dalloc(&n->wpart, wp)) != hipSuccess) return oom(e);
  const int64_t npx = (int64_t)B * n->N * n->N;
  if ((e = dalloc(&n->x0buf, (size_t)npx)) != hipSuccess) return oom(e);
  if ((e = dalloc(&n->hpart, cnn::head_part_doubles(n->c[0], npx))) != hipSuccess) return oom(e);
  if ((e = dalloc(&n->d_loss, 1)) != hipSuccess) return oom(e);
  if ((e = hipHostMalloc((void**)&n->h_loss, sizeof(double), hipHostMallocDefault)) != hipSuccess)
    return oom(e);
  if ((e = cnn::launch_zero(n->p, n->n_params, n->st)) != hipSuccess) return oom(e);
  if ((e = cast_all(n)) != hipSuccess) return oom(e);
  if ((e = hipStreamSynchronize(n->st)) != hipSuccess) return oom(e);
  n->valid = true;
  *out = n;
  return SLIM_OK;
}

int64_t slim_cnn_num_params(const slim_cnn* n) { return n ? n->n_params : 0; }

double slim_cnn_forward_flops(const slim_cnn* n) {
  if (!n) return 0.0;
  double f = 0.0;
  for (int li = 0; li < (int)n->layers.size(); ++li) {
    const Layer& ly = n->layers[li];
    int H = n->N;
    for (int l = 0; l < n->L; ++l)
      if (li == n->e_a(l) || li == n->e_b(l) ||
          (l < n->L - 1 && (li == n->u_(l) || li == n->d_a(l) || li == n->d_b(l))))
        H = n->H(l);
    f += 2.0 * 9.0 * ly.Cin * ly.Cout * (double)H * H;
  }
  return f + 2.0 * (n->c[0] + 1) * (double)n->N * n->N;
}

slim_status slim_cnn_set_params(slim_cnn* n, const float* host, int64_t count) {
  if (!n || !host) return cnn_fail(SLIM_EINVAL, "net or host is NULL");
  if (count != n->n_params) return cnn_fail(SLIM_EINVAL, "parameter count mismatch");
  bool finite = true;
  for (int64_t i = 0; i < count && finite; ++i) finite = std::isfinite(host[i]);
  CNN_TRY(hipMemcpyAsync(n->p, host, sizeof(float) * count, hipMemcpyHostToDevice, n->st));
  CNN_TRY(cnn::launch_zero(n->m, count, n->st));
  CNN_TRY(cnn::launch_zero(n->v, count, n->st));
  CNN_TRY(cast_all(n));
  CNN_TRY(hipStreamSynchronize(n->st));
  n->valid = finite;
  n->t = 0;
  n->have_grad = false;
  return SLIM_OK;
}

slim_status slim_cnn_get_params(slim_cnn* n, float* host, int64_t count) {
  if (!n || !host) return cnn_fail(SLIM_EINVAL, "net or host is NULL");
  if (count != n->n_params) return cnn_fail(SLIM_EINVAL, "parameter count mismatch");
  CNN_TRY(hipMemcpyAsync(host, n->p, sizeof(float) * count, hipMemcpyDeviceToHost, n->st));
  CNN_TRY(hipStreamSynchronize(n->st));
  return SLIM_OK;
}

slim_status slim_cnn_forward(slim_cnn* n, const float* u, float* x0, int B) {
  if (!n || !u || !x0) return cnn_fail(SLIM_EINVAL, "net, u or x0 is NULL");
  slim_status s = check_batch(n, B);
  if (s != SLIM_OK) return s;
  if (!n->valid) return cnn_fail(SLIM_ESTATE, "network parameters are not finite");
  CNN_TRY(forward(n, u, x0, B));
  return SLIM_OK;
}

slim_status slim_cnn_loss_grad(slim_cnn* n, const float* u, const float* target, int B,
                               double* loss, float* grad_host) {
  if (!n || !u || !target) return cnn_fail(SLIM_EINVAL, "net, u or target is NULL");
  slim_status s = check_batch(n, B);
  if (s != SLIM_OK) return s;
  if (!n->valid) return cnn_fail(SLIM_ESTATE, "network parameters are not finite");
  CNN_TRY(forward(n, u, n->x0buf, B));
  CNN_TRY(backward(n, u, target, B));
  n->have_grad = true;
  if (loss) {
    CNN_TRY(hipMemcpyAsync(n->h_loss, n->d_loss, sizeof(double), hipMemcpyDeviceToHost, n->st));
  }
  if (grad_host) {
    CNN_TRY(hipMemcpyAsync(grad_host, n->g, sizeof(float) * n->n_params, hipMemcpyDeviceToHost,
                           n->st));
  }
  if (loss || grad_host) CNN_TRY(hipStreamSynchronize(n->st));
  if (loss) *loss = *n->h_loss;
  return SLIM_OK;
}

slim_status slim_cnn_adam(slim_cnn* n, double lr, double beta1, double beta2, double eps) {
  if (!n) return cnn_fail(SLIM_EINVAL, "net is NULL");
  if (!(lr > 0.0) || !(beta1 >= 0.0 && beta1 < 1.0) || !(beta2 >= 0.0 && beta2 < 1.0) ||
      !(eps > 0.0))
    return cnn_fail(SLIM_EINVAL, "Adam hyper-parameters out of range");
  if (!n->have_grad) return cnn_fail(SLIM_ESTATE, "no gradient (call slim_cnn_loss_grad)");
  n->t += 1;
  const double c1 = 1.0 - std::pow(beta1, n->t), c2 = 1.0 - std::pow(beta2, n->t);
  const float lr_t = (float)(lr * std::sqrt(c2) / c1), eps_t = (float)(eps * std::sqrt(c2));
  CNN_TRY(cnn::launch_adam(n->p, n->g, n->m, n->v, n->n_params, (float)beta1, (float)beta2, lr_t,
                           eps_t, n->st));
  CNN_TRY(cast_all(n));
  return SLIM_OK;
}

void slim_cnn_destroy(slim_cnn* n) { delete n; }

}  // extern "C"
