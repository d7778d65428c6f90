// Matrix-free Joseph projectors for gfx950.
//
// Forward (ray-driven, LDS bands): the image is cut into bands of H rows
// (row-stepping angles) or H rows of its transpose (column-stepping angles,
// i.e. H image columns), H*(N+4) floats <= 64 KB.  A workgroup owns a group
// of consecutive bands and a chunk of angles of one orientation; it streams
// its bands through LDS (zero-padded by two pixels on each side, so no
// bounds checks in the inner loop) and every lane walks up to 8 rays across
// them, interpolating linearly between the two pixels nearest the crossing
// point (Joseph), accumulating in float64.  Per-group partial sums are
// combined by a second kernel in a fixed order (deterministic, no atomics).
// Workgroups are numbered so that each XCD works on a contiguous range of
// band groups and its L2 holds only its slice of the image.
//
// Back (pixel-driven gather): a workgroup owns a 16 x 64 pixel tile and
// stages, for every angle of the list, the segment of ray values its tile
// touches (scaled by h/d) in LDS; each lane gathers two rays per angle for
// four consecutive pixels of a row.  No atomics; the optional fused update
// writes x -= s, the transposed image, and per-workgroup float64 partial
// norms.  Both projectors evaluate the same closed-form weights and agree to
// float32 rounding of the weights.
#include "slim_internal.h"
#include "pcg.h"

#include <algorithm>

namespace slim {

namespace {

// ---------------------------------------------------------------- forward
constexpr int kFT = 512;      // threads per forward workgroup
constexpr int kFItems = 4;    // rays per lane
constexpr int kPad = 4;       // zero columns on each side of a band row (keeps rows 16B-aligned)
// float4 per lane per band: H * N / 4 <= 16384 / 4 = 8 * kFT (eight prefetch registers)

struct FwdPlan {
  int n;          // entries (= output rows)
  int n_row;      // entries 0..n_row-1 are row-stepping angles
  int ch;         // angles per chunk
  int n_chunks;   // row-stepping chunks first
  int H, G;       // rows per band, bands per group
  int n_groups;
  int items;      // rays per lane (template argument of the band kernel)
  short id[kMaxList];
  short slot[kMaxList];
};

// bf16 storage (upper half of a float32, round-to-nearest-even on store)
__device__ __forceinline__ float bf2f(uint16_t b) { return __uint_as_float((uint32_t)b << 16); }
__device__ __forceinline__ uint16_t f2bf(float f) {
  uint32_t u = __float_as_uint(f);
  if ((u & 0x7fffffffu) > 0x7f800000u) return (uint16_t)((u >> 16) | 0x40u);  // quiet NaN
  u += 0x7fffu + ((u >> 16) & 1u);
  return (uint16_t)(u >> 16);
}
__device__ __forceinline__ float tof(float v) { return v; }
__device__ __forceinline__ float tof(uint16_t v) { return bf2f(v); }
// four consecutive pixels starting at element 4*i
__device__ __forceinline__ float4 load4(const float* p, int i) {
  return reinterpret_cast<const float4*>(p)[i];
}
__device__ __forceinline__ float4 load4(const uint16_t* p, int i) {
  const uint2 u = reinterpret_cast<const uint2*>(p)[i];
  return make_float4(__uint_as_float(u.x << 16), __uint_as_float(u.x & 0xffff0000u),
                     __uint_as_float(u.y << 16), __uint_as_float(u.y & 0xffff0000u));
}

__device__ __forceinline__ void chunk_range(const FwdPlan& pl, int c, int& e0, int& e1, bool& colm) {
  const int nrc = (pl.n_row + pl.ch - 1) / pl.ch;
  if (c < nrc) {
    e0 = c * pl.ch;
    e1 = min(pl.n_row, e0 + pl.ch);
    colm = false;
  } else {
    e0 = pl.n_row + (c - nrc) * pl.ch;
    e1 = min(pl.n, e0 + pl.ch);
    colm = true;
  }
}

template <int IT, typename IMG>
__global__ __launch_bounds__(kFT, 2) void fwd_band_kernel(const AngleGeom* __restrict__ geom, int N,
                                                          int R, FwdPlan pl,
                                                          const IMG* __restrict__ img,
                                                          const IMG* __restrict__ imgT,
                                                          float* __restrict__ partial,
                                                          const int* __restrict__ stop) {
  if (stop && stop[kCtlDone]) return;
  extern __shared__ float band[];
  const int W = N + 2 * kPad;
  // XCD-aware numbering: consecutive positions live on one XCD
  const int total = pl.n_groups * pl.n_chunks;
  const int per_xcd = gridDim.x >> 3;
  const int pos = (blockIdx.x & 7) * per_xcd + (blockIdx.x >> 3);
  if (pos >= total) return;
  const int grp = pos / pl.n_chunks;
  const int chunk = pos % pl.n_chunks;
  int e0, e1;
  bool colm;
  chunk_range(pl, chunk, e0, e1, colm);
  const int nitems = (e1 - e0) * R;
  const IMG* src = colm ? imgT : img;
  const double half = 0.5 * (N - 1);
  const double off = 0.5 * (R - 1);
  const int kg = grp * pl.G * pl.H;

  // Ray position along the minor axis in 32.32 fixed point: P = pos * 2^32
  // at row k is P0 + k * S (pos: 0-based pixel index shifted by kPad).
  // Rounding P0 and S costs at most (k+1) * 2^-33 < 1.2e-7 pixel at k = 1023.
  // Each wavefront walks, per ray slot, the union of its 64 rays' row ranges
  // (a wave-uniform loop); a lane outside its own ray's range reads the zero
  // pads (its index is clamped into [0, W-2]) and adds nothing.
  int64_t P0[IT], S[IT];
  double acc[IT];
  int wlo[IT], whi[IT];
#pragma unroll
  for (int q = 0; q < IT; ++q) {
    const int item = threadIdx.x + q * kFT;
    acc[q] = 0.0;
    P0[q] = 0;  // index 0: pad column
    S[q] = 0;
    int klo = N, khi = -1;
    if (item < nitems) {
      const int e = e0 + item / R;
      const int t = item % R;
      const AngleGeom g = geom[pl.id[e]];
      const double cm = colm ? g.c : g.s;   // coefficient of the major coordinate
      const double cn = colm ? g.s : g.c;   // of the minor one, |cn| = d
      const double inv = 1.0 / cn;
      const double n1 = -cm * inv;          // pos(k) = p0 + k * n1
      const double p0 = ((double)t - off) * inv + half + kPad - half * n1;
      // rows with pos - kPad in [-1.5, N + 0.5] hold every contributing row
      const double lo_p = kPad - 1.5, hi_p = N + kPad + 0.5;
      double lo = 0.0, hi = N - 1;
      if (n1 != 0.0) {
        const double ma = (lo_p - p0) / n1, mb = (hi_p - p0) / n1;
        lo = fmax(lo, ceil(fmin(ma, mb)));
        hi = fmin(hi, floor(fmax(ma, mb)));
      } else if (p0 < lo_p || p0 > hi_p) {
        lo = 1.0;
        hi = 0.0;
      }
      if (lo <= hi) {
        klo = (int)lo;
        khi = (int)hi;
      }
      P0[q] = __double2ll_rn(p0 * 4294967296.0);
      S[q] = __double2ll_rn(n1 * 4294967296.0);
    }
    for (int o = 32; o > 0; o >>= 1) {
      klo = min(klo, __shfl_xor(klo, o, 64));
      khi = max(khi, __shfl_xor(khi, o, 64));
    }
    wlo[q] = __builtin_amdgcn_readfirstlane(klo);
    whi[q] = __builtin_amdgcn_readfirstlane(khi);
  }

  {  // the zero pads are written once; band loads never touch them
    for (int e = threadIdx.x; e < pl.H * 2 * kPad; e += kFT) {
      const int r = e / (2 * kPad), c = e % (2 * kPad);
      band[r * W + (c < kPad ? c : N + c)] = 0.f;
    }
  }
  // Bands are software-pipelined: the next band's rows are fetched into
  // eight named registers (16-byte loads) while the current band is used.
  const bool vec = (N & 3) == 0;
  const int n4 = N >> 2;
  float4 pf0, pf1, pf2, pf3, pf4, pf5, pf6, pf7;
#define SLIM_PF_LOAD(kb_)                                                       \
  do {                                                                          \
    const IMG* s4 = src + (size_t)(kb_) * N;                                    \
    const int lim = min(pl.H, N - (kb_)) * n4 - 1;                               \
    const int t0 = (int)threadIdx.x;                                            \
    pf0 = load4(s4, min(t0 + 0 * kFT, lim));                                    \
    pf1 = load4(s4, min(t0 + 1 * kFT, lim));                                    \
    pf2 = load4(s4, min(t0 + 2 * kFT, lim));                                    \
    pf3 = load4(s4, min(t0 + 3 * kFT, lim));                                    \
    pf4 = load4(s4, min(t0 + 4 * kFT, lim));                                    \
    pf5 = load4(s4, min(t0 + 5 * kFT, lim));                                    \
    pf6 = load4(s4, min(t0 + 6 * kFT, lim));                                    \
    pf7 = load4(s4, min(t0 + 7 * kFT, lim));                                    \
  } while (0)
#define SLIM_PF_STORE1(u, v)                                                    \
  do {                                                                          \
    const int e = (int)threadIdx.x + (u) * kFT;                                 \
    const int r = e / n4, c4 = e - r * n4;                                      \
    if (e < lim) *reinterpret_cast<float4*>(band + r * W + kPad + 4 * c4) = (v); \
  } while (0)
  if (vec && kg < N) SLIM_PF_LOAD(kg);
  for (int bb = 0; bb < pl.G; ++bb) {
    const int kb = kg + bb * pl.H;
    if (kb >= N) break;
    const int hb = min(pl.H, N - kb);
    __syncthreads();
    if (vec) {
      const int lim = hb * n4;
      SLIM_PF_STORE1(0, pf0);
      SLIM_PF_STORE1(1, pf1);
      SLIM_PF_STORE1(2, pf2);
      SLIM_PF_STORE1(3, pf3);
      SLIM_PF_STORE1(4, pf4);
      SLIM_PF_STORE1(5, pf5);
      SLIM_PF_STORE1(6, pf6);
      SLIM_PF_STORE1(7, pf7);
    } else {
      for (int r = 0; r < hb; ++r)
        for (int c = threadIdx.x; c < N; c += kFT)
          band[r * W + kPad + c] = tof(src[(size_t)(kb + r) * N + c]);
    }
    __syncthreads();
    const int kbn = kb + pl.H;
    if (vec && bb + 1 < pl.G && kbn < N) SLIM_PF_LOAD(kbn);
#pragma unroll
    for (int q = 0; q < IT; ++q) {
      const int k0 = max(wlo[q], kb), k1 = min(whi[q], kb + hb - 1);
      if (k0 > k1) continue;  // wave-uniform
      int64_t P = P0[q] + (int64_t)k0 * S[q];
      const float* row = band + (k0 - kb) * W;
      float a32 = 0.f;
      for (int k = k0; k <= k1; ++k) {
        const int qi = min(max((int)(P >> 32), 0), W - 2);
        const float phi = (float)(uint32_t)P * 2.3283064365386963e-10f;
        const float v0 = row[qi], v1 = row[qi + 1];
        a32 += fmaf(phi, v1 - v0, v0);
        P += S[q];
        row += W;
      }
      acc[q] += (double)a32;
    }
  }
#undef SLIM_PF_LOAD
#undef SLIM_PF_STORE1
#pragma unroll
  for (int q = 0; q < IT; ++q) {
    const int item = threadIdx.x + q * kFT;
    if (item < nitems) {
      const int e = e0 + item / R;
      const int t = item % R;
      partial[((size_t)grp * pl.n + pl.slot[e]) * R + t] = (float)acc[q];
    }
  }
}

// out[s][t] = (h/d) sum_groups partial - sub; optional CG tail q = out + lam*pd
// with per-workgroup partial dot <pd, q>.
template <typename SUB>
__global__ __launch_bounds__(256) void fwd_reduce_kernel(const AngleGeom* __restrict__ geom, int R,
                                                         AngleList ids, int n_groups,
                                                         const float* __restrict__ partial,
                                                         const SUB* __restrict__ sub,
                                                         float* __restrict__ out32,
                                                         double* __restrict__ out64,
                                                         const double* __restrict__ pd, double lam,
                                                         double* __restrict__ dots,
                                                         const int* __restrict__ stop) {
  if (stop && stop[kCtlDone]) return;
  __shared__ double sh[4];
  const int o = blockIdx.x * 256 + threadIdx.x;
  const int n = ids.n * R;
  double d = 0.0;
  if (o < n) {
    const int s = o / R, t = o % R;
    const int ang = ids.id[s];
    const float* pp = partial + (size_t)s * R + t;
    const size_t gs = (size_t)ids.n * R;
    double v = 0.0;
    int g = 0;
    for (; g + 4 <= n_groups; g += 4) {
      const float a = pp[g * gs], b = pp[(g + 1) * gs], c = pp[(g + 2) * gs], e = pp[(g + 3) * gs];
      v += (double)a;
      v += (double)b;
      v += (double)c;
      v += (double)e;
    }
    for (; g < n_groups; ++g) v += (double)pp[g * gs];
    const double hd = (double)geom[ang].hd;
    v *= hd;
    if (sub) v -= (double)tof(sub[(size_t)ang * R + t]);
    if (pd) {
      v = fma(lam, pd[o], v);
      d = pd[o] * v;
    }
    if (out32) out32[o] = (float)v;
    if (out64) out64[o] = v;
  }
  if (dots) {
    for (int w = 32; w > 0; w >>= 1) d += __shfl_down(d, w, 64);
    if ((threadIdx.x & 63) == 0) sh[threadIdx.x >> 6] = d;
    __syncthreads();
    if (threadIdx.x == 0) dots[blockIdx.x] = sh[0] + sh[1] + sh[2] + sh[3];
  }
}

// Launch plan: angles grouped by orientation into chunks, image bands into
// groups, with n_chunks * n_groups <= 2 * (number of CUs) so that a launch is
// a single round of resident workgroups (two per CU, bounded by LDS).
FwdPlan make_plan(const AngleGeom* h_geom, int N, int R, const AngleList& ids, int n_cu) {
  FwdPlan pl;
  pl.n = ids.n;
  int k = 0;
  for (int pass = 0; pass < 2; ++pass)
    for (int s = 0; s < ids.n; ++s)
      if ((h_geom[ids.id[s]].colmajor != 0) == (pass == 1)) {
        pl.id[k] = (short)ids.id[s];
        pl.slot[k] = (short)s;
        ++k;
      }
  pl.n_row = 0;
  for (int s = 0; s < ids.n; ++s) pl.n_row += h_geom[ids.id[s]].colmajor ? 0 : 1;
  pl.ch = std::max(1, std::min(kFItems * kFT / R, ids.n));
  pl.items = (pl.ch * R + kFT - 1) / kFT;
  pl.n_chunks = (pl.n_row + pl.ch - 1) / pl.ch + (ids.n - pl.n_row + pl.ch - 1) / pl.ch;
  pl.H = std::max(1, std::min(N, 16384 / (N + 2 * kPad)));
  const int nbands = (N + pl.H - 1) / pl.H;
  const int slots = 2 * std::max(1, n_cu);
  int want = std::max(1, std::min(slots / pl.n_chunks, nbands));
  pl.G = (nbands + want - 1) / want;
  pl.n_groups = (nbands + pl.G - 1) / pl.G;
  return pl;
}

// ------------------------------------------------------------------- back
constexpr int kBH = 16, kBW = 64;   // tile rows, columns
constexpr int kBPX = 4;             // consecutive pixels per lane
constexpr int kBAng = 64;           // angles staged per pass
constexpr int kSeg = 72;            // LDS stride of one angle's ray segment

__device__ __forceinline__ double wave_sum(double v) {
  for (int o = 32; o > 0; o >>= 1) v += __shfl_down(v, o, 64);
  return v;
}

template <typename VT>
__global__ __launch_bounds__(256) void back_kernel(const AngleGeom* __restrict__ geom, int N, int R,
                                                   AngleList ids, const VT* __restrict__ v,
                                                   float* __restrict__ out, float* __restrict__ x,
                                                   float* __restrict__ xT,
                                                   const float* __restrict__ x_true,
                                                   double* __restrict__ partials, int mode,
                                                   const int* __restrict__ stop,
                                                   uint16_t* __restrict__ xs,
                                                   uint16_t* __restrict__ xsT) {
  if (stop && stop[kCtlDone]) return;
  __shared__ float seg[kBAng * kSeg];
  __shared__ int tmin[kBAng];
  __shared__ float tile[kBH][kBW + 1];
  __shared__ double wred[4][3];
  const int tx = threadIdx.x & 15;       // 16 lanes x 4 pixels = 64 columns
  const int ty = threadIdx.x >> 4;       // 16 rows
  const int i0 = blockIdx.y * kBH, j0 = blockIdx.x * kBW;
  const int i = i0 + ty;
  const int jb = j0 + kBPX * tx;
  const double half = 0.5 * (N - 1);
  // detector coordinates are shifted by kTOff (>= every |jj c + ii s|), so
  // they are positive and float->int truncation is floor
  const int kTOff = 2 * N + 8;
  const double off = 0.5 * (R - 1) + kTOff;
  const double ii = (double)i - half;
  // nominal tile corners (pixel centres) bound every pixel the lanes evaluate
  const double ci0 = (double)i0 - half, ci1 = (double)(i0 + kBH - 1) - half;
  const double cj0 = (double)j0 - half, cj1 = (double)(j0 + kBW - 1) - half;
  float s[kBPX] = {0.f, 0.f, 0.f, 0.f};
  for (int a0 = 0; a0 < ids.n; a0 += kBAng) {
    const int na = min(kBAng, ids.n - a0);
    __syncthreads();
    if ((int)threadIdx.x < na) {
      const AngleGeom g = geom[ids.id[a0 + threadIdx.x]];
      const double t00 = det_coord(g, ci0, cj0, off), t01 = det_coord(g, ci0, cj1, off);
      const double t10 = det_coord(g, ci1, cj0, off), t11 = det_coord(g, ci1, cj1, off);
      tmin[threadIdx.x] = (int)floor(fmin(fmin(t00, t01), fmin(t10, t11))) - 1;
    }
    __syncthreads();
    for (int e = threadIdx.x; e < na * kSeg; e += 256) {
      const int a = e / kSeg, u = e % kSeg;
      const int t = tmin[a] + u - kTOff;
      const AngleGeom& g = geom[ids.id[a0 + a]];
      seg[e] = (t >= 0 && t < R) ? g.hd * (float)v[(size_t)(a0 + a) * R + t] : 0.f;
    }
    __syncthreads();
    if (i < N) {
      for (int a = 0; a < na; ++a) {
        const AngleGeom g = geom[ids.id[a0 + a]];
        const double Ti = fma(ii, g.s, off);
        const float* sa = seg + a * kSeg - tmin[a];
        const float invd = g.invd, c1 = 1.f - g.invd;
#pragma unroll
        for (int q = 0; q < kBPX; ++q) {
          const double t = fma((double)(jb + q) - half, g.c, Ti);
          const int t0 = (int)t;                       // t > 0: floor
          const float f = (float)(t - (double)t0);     // distance to ray t0
          const float w0 = fmaxf(0.f, fmaf(-f, invd, 1.f));   // 1 - f/d
          const float w1 = fmaxf(0.f, fmaf(f, invd, c1));     // 1 - (1-f)/d
          s[q] = fmaf(w0, sa[t0], fmaf(w1, sa[t0 + 1], s[q]));
        }
      }
    }
  }
  const bool full = (i < N) && (jb + kBPX - 1 < N);
  if (mode == 0) {
    if (full && (N & 3) == 0) {
      *reinterpret_cast<float4*>(out + (size_t)i * N + jb) = make_float4(s[0], s[1], s[2], s[3]);
    } else if (i < N) {
      for (int q = 0; q < kBPX; ++q)
        if (jb + q < N) out[(size_t)i * N + jb + q] = s[q];
    }
    if (xT) {
      __syncthreads();
#pragma unroll
      for (int q = 0; q < kBPX; ++q) tile[ty][kBPX * tx + q] = s[q];
      __syncthreads();
      for (int e = threadIdx.x; e < kBH * kBW; e += 256) {
        const int jl = e / kBH, il = e % kBH;
        if (j0 + jl < N && i0 + il < N) xT[(size_t)(j0 + jl) * N + i0 + il] = tile[il][jl];
      }
    }
    return;
  }
  double ss = 0.0, xx = 0.0, ee = 0.0;
  float xn[kBPX] = {0.f, 0.f, 0.f, 0.f};
  if (i < N) {
#pragma unroll
    for (int q = 0; q < kBPX; ++q) {
      if (jb + q < N) {
        const size_t p = (size_t)i * N + jb + q;
        xn[q] = x[p] - s[q];
        x[p] = xn[q];
        if (xs) xs[p] = f2bf(xn[q]);
        ss += (double)s[q] * (double)s[q];
        xx += (double)xn[q] * (double)xn[q];
        if (x_true) {
          const double e = (double)xn[q] - (double)x_true[p];
          ee += e * e;
        }
      }
    }
  }
  if (xT || xsT) {
    __syncthreads();
#pragma unroll
    for (int q = 0; q < kBPX; ++q) tile[ty][kBPX * tx + q] = xn[q];
    __syncthreads();
    for (int e = threadIdx.x; e < kBH * kBW; e += 256) {
      const int jl = e / kBH, il = e % kBH;
      if (j0 + jl < N && i0 + il < N) {
        const size_t o = (size_t)(j0 + jl) * N + i0 + il;
        if (xT) xT[o] = tile[il][jl];
        if (xsT) xsT[o] = f2bf(tile[il][jl]);
      }
    }
  }
  ss = wave_sum(ss);
  xx = wave_sum(xx);
  ee = wave_sum(ee);
  const int w = threadIdx.x >> 6;
  if ((threadIdx.x & 63) == 0) {
    wred[w][0] = ss;
    wred[w][1] = xx;
    wred[w][2] = ee;
  }
  __syncthreads();
  if (threadIdx.x < 3) {
    const double r = wred[0][threadIdx.x] + wred[1][threadIdx.x] + wred[2][threadIdx.x] +
                     wred[3][threadIdx.x];
    partials[(size_t)3 * (blockIdx.y * gridDim.x + blockIdx.x) + threadIdx.x] = r;
  }
}

__global__ __launch_bounds__(256) void reduce3_kernel(const double* __restrict__ partials, int n,
                                                      double* __restrict__ out) {
  __shared__ double red[3][256];
  double a0 = 0.0, a1 = 0.0, a2 = 0.0;
  for (int k = threadIdx.x; k < n; k += 256) {
    a0 += partials[3 * (size_t)k + 0];
    a1 += partials[3 * (size_t)k + 1];
    a2 += partials[3 * (size_t)k + 2];
  }
  red[0][threadIdx.x] = a0;
  red[1][threadIdx.x] = a1;
  red[2][threadIdx.x] = a2;
  __syncthreads();
  for (int sz = 128; sz > 0; sz >>= 1) {
    if ((int)threadIdx.x < sz) {
      red[0][threadIdx.x] += red[0][threadIdx.x + sz];
      red[1][threadIdx.x] += red[1][threadIdx.x + sz];
      red[2][threadIdx.x] += red[2][threadIdx.x + sz];
    }
    __syncthreads();
  }
  if (threadIdx.x < 3) out[threadIdx.x] = red[threadIdx.x][0];
}

constexpr int kTile = 16;

// dst = src^T (float32, optional); bf16 copies of src and of src^T (optional)
__global__ __launch_bounds__(256) void transpose_kernel(const float* __restrict__ src,
                                                        float* __restrict__ dst, int N,
                                                        uint16_t* __restrict__ bs,
                                                        uint16_t* __restrict__ bsT) {
  __shared__ float t[kTile][kTile + 1];
  const int tx = threadIdx.x & (kTile - 1), ty = threadIdx.x / kTile;
  const int i = blockIdx.y * kTile + ty, j = blockIdx.x * kTile + tx;
  if (i < N && j < N) {
    const float v = src[(size_t)i * N + j];
    t[ty][tx] = v;
    if (bs) bs[(size_t)i * N + j] = f2bf(v);
  }
  __syncthreads();
  const int jt = blockIdx.x * kTile + ty, it = blockIdx.y * kTile + tx;
  if (jt < N && it < N) {
    if (dst) dst[(size_t)jt * N + it] = t[tx][ty];
    if (bsT) bsT[(size_t)jt * N + it] = f2bf(t[tx][ty]);
  }
}

}  // namespace

size_t forward_partial_floats(int N, int R, int max_list) {
  const int H = std::max(1, std::min(N, 16384 / (N + 2 * kPad)));
  const size_t nbands = (size_t)(N + H - 1) / H;
  return nbands * (size_t)max_list * (size_t)R;
}

int forward_dot_parts(int n_out) { return (n_out + 255) / 256; }

static int g_num_cu = 0;

static int num_cu() {
  if (g_num_cu == 0) {
    int dev = 0, n = 0;
    if (hipGetDevice(&dev) == hipSuccess &&
        hipDeviceGetAttribute(&n, hipDeviceAttributeMultiprocessorCount, dev) == hipSuccess && n > 0)
      g_num_cu = n;
    else
      g_num_cu = 256;
  }
  return g_num_cu;
}

template <typename IMG>
static void launch_band(int items, dim3 grid, size_t lds, hipStream_t st, const AngleGeom* geom,
                        int N, int R, const FwdPlan& pl, const IMG* img, const IMG* imgT,
                        float* partial, const int* stop) {
  switch (items) {
    case 1:
      hipLaunchKernelGGL((fwd_band_kernel<1, IMG>), grid, dim3(kFT), lds, st, geom, N, R, pl, img,
                         imgT, partial, stop);
      break;
    case 2:
      hipLaunchKernelGGL((fwd_band_kernel<2, IMG>), grid, dim3(kFT), lds, st, geom, N, R, pl, img,
                         imgT, partial, stop);
      break;
    case 3:
      hipLaunchKernelGGL((fwd_band_kernel<3, IMG>), grid, dim3(kFT), lds, st, geom, N, R, pl, img,
                         imgT, partial, stop);
      break;
    default:
      hipLaunchKernelGGL((fwd_band_kernel<4, IMG>), grid, dim3(kFT), lds, st, geom, N, R, pl, img,
                         imgT, partial, stop);
      break;
  }
}

hipError_t launch_forward(const AngleGeom* geom, const AngleGeom* h_geom, int N, int R,
                          const AngleList& ids, const void* img, const void* imgT, int img_bf16,
                          const void* sub, int sub_bf16, float* out32, double* out64,
                          float* partial, const double* pd, double lam, double* dots,
                          const int* stop, hipStream_t st) {
  if (ids.n <= 0) return hipSuccess;
  const FwdPlan pl = make_plan(h_geom, N, R, ids, num_cu());
  const int total = pl.n_groups * pl.n_chunks;
  const int nwg = (total + 7) / 8 * 8;
  const size_t lds = (size_t)pl.H * (N + 2 * kPad) * sizeof(float);
  if (img_bf16)
    launch_band(pl.items, dim3(nwg), lds, st, geom, N, R, pl, (const uint16_t*)img,
                (const uint16_t*)imgT, partial, stop);
  else
    launch_band(pl.items, dim3(nwg), lds, st, geom, N, R, pl, (const float*)img,
                (const float*)imgT, partial, stop);
  const int n = ids.n * R;
  const dim3 rg((n + 255) / 256);
  if (sub_bf16)
    hipLaunchKernelGGL(fwd_reduce_kernel<uint16_t>, rg, dim3(256), 0, st, geom, R, ids, pl.n_groups,
                       partial, (const uint16_t*)sub, out32, out64, pd, lam, dots, stop);
  else
    hipLaunchKernelGGL(fwd_reduce_kernel<float>, rg, dim3(256), 0, st, geom, R, ids, pl.n_groups,
                       partial, (const float*)sub, out32, out64, pd, lam, dots, stop);
  return hipGetLastError();
}

int back_num_workgroups(int N) { return ((N + kBW - 1) / kBW) * ((N + kBH - 1) / kBH); }

hipError_t launch_back(const AngleGeom* geom, int N, int R, const AngleList& ids,
                       const float* v32, const double* v64, float* out, float* x, float* xT,
                       const float* x_true, double* partials, int mode, const int* stop,
                       uint16_t* xs, uint16_t* xsT, hipStream_t st) {
  dim3 grid((N + kBW - 1) / kBW, (N + kBH - 1) / kBH);
  if (v64) {
    hipLaunchKernelGGL(back_kernel<double>, grid, dim3(256), 0, st, geom, N, R, ids, v64, out, x,
                       xT, x_true, partials, mode, stop, xs, xsT);
  } else {
    hipLaunchKernelGGL(back_kernel<float>, grid, dim3(256), 0, st, geom, N, R, ids, v32, out, x,
                       xT, x_true, partials, mode, stop, xs, xsT);
  }
  return hipGetLastError();
}

hipError_t launch_reduce3(const double* partials, int n, double* out, hipStream_t st) {
  hipLaunchKernelGGL(reduce3_kernel, dim3(1), dim3(256), 0, st, partials, n, out);
  return hipGetLastError();
}

hipError_t launch_transpose(const float* src, float* dst, int N, uint16_t* bs, uint16_t* bsT,
                            hipStream_t st) {
  const int t = (N + kTile - 1) / kTile;
  hipLaunchKernelGGL(transpose_kernel, dim3(t, t), dim3(256), 0, st, src, dst, N, bs, bsT);
  return hipGetLastError();
}

}  // namespace slim
