// Kernels of the warm-start CNN for gfx950.
//
// 3x3 convolutions are implicit GEMMs on v_mfma_f32_16x16x32_bf16 (M =
// pixels, N = output channels, K = 9 taps x input channels).  A wavefront
// owns 64 output pixels x 32 output channels (4 x 2 MFMA tiles) and reads its
// operands straight from L1/L2: in NHWC the 8 consecutive channels a lane
// supplies are one 16-byte load.  MFMA operand layout (lane l = 16 q + r):
// A holds row r, k = 8q..8q+7; B holds column r, k = 8q..8q+7; accumulator
// e of lane l is D[4q + e][r].
//
// On grids of at least 32 x 32 the operands are staged in LDS instead
// (conv3x3_lds_kernel below).
//
// Weight gradients contract over pixels, the strided dimension of NHWC, so
// their workgroups stage 64-pixel chunks of dz and of the shifted input
// through LDS transposed (pixel-contiguous rows) and write split-K partials
// that a second kernel sums in a fixed order (bitwise reproducible).
#include <algorithm>

#include "cnn_internal.h"

namespace slim {
namespace cnn {
namespace {

typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef float f32x4 __attribute__((ext_vector_type(4)));
typedef unsigned int u32x4 __attribute__((ext_vector_type(4)));

__device__ __forceinline__ float bf2f(uint16_t h) { return __uint_as_float((uint32_t)h << 16); }

// float -> bf16, round to nearest even (NaN stays NaN)
__device__ __forceinline__ uint16_t f2bf(float f) {
  uint32_t u = __float_as_uint(f);
  if ((u & 0x7fffffffu) > 0x7f800000u) return 0x7fc0;
  u += 0x7fffu + ((u >> 16) & 1u);
  return (uint16_t)(u >> 16);
}

__device__ __forceinline__ bf16x8 ld8(const uint16_t* p) {
  return __builtin_bit_cast(bf16x8, *reinterpret_cast<const u32x4*>(p));
}

__device__ __forceinline__ bf16x8 zero8() {
  u32x4 z = {0u, 0u, 0u, 0u};
  return __builtin_bit_cast(bf16x8, z);
}

// Blocks are dispatched round-robin over the 8 XCDs; this numbering gives
// consecutive logical blocks (neighbouring pixel tiles, which share input
// rows) to one XCD and its L2.  gridDim.x must be a multiple of 8.
__device__ __forceinline__ int64_t xcd_block() {
  return (int64_t)(blockIdx.x & 7) * (gridDim.x >> 3) + (blockIdx.x >> 3);
}

unsigned grid8(int64_t blocks) { return (unsigned)((blocks + 7) / 8 * 8); }

// ------------------------------------------------------------ convolution
constexpr int kCW = 4;  // wavefronts per conv workgroup

__global__ __launch_bounds__(64 * kCW) void conv3x3_kernel(ConvArgs a, int64_t n_wave_tiles) {
  const int lane = threadIdx.x & 63;
  const int64_t wt = xcd_block() * kCW + (threadIdx.x >> 6);
  if (wt >= n_wave_tiles) return;
  const int nco = a.Cout >> 5;
  const int cot = (int)(wt % nco);
  const int64_t pt = wt / nco;
  const int H = a.H, HW = H * H;
  const int Hin = a.up ? (H >> 1) : H;
  const int r = lane & 15, q = lane >> 4;

  int py[4], px[4];
  int64_t img[4];
#pragma unroll
  for (int i = 0; i < 4; ++i) {
    const int64_t P = pt * 64 + 16 * i + r;
    const int64_t n = P / HW;
    const int rem = (int)(P - n * HW);
    py[i] = rem / H;
    px[i] = rem - py[i] * H;
    img[i] = n * Hin * Hin;
  }
  const uint16_t* wrow[2];
#pragma unroll
  for (int j = 0; j < 2; ++j) wrow[j] = a.w + (size_t)(cot * 32 + 16 * j + r) * 9 * a.Cin + 8 * q;

  f32x4 acc[4][2];
#pragma unroll
  for (int i = 0; i < 4; ++i)
#pragma unroll
    for (int j = 0; j < 2; ++j) acc[i][j] = f32x4{0.f, 0.f, 0.f, 0.f};

  for (int tap = 0; tap < 9; ++tap) {
    const int dy = tap / 3 - 1, dx = tap % 3 - 1;
    const uint16_t* src[4];
    bool ok[4];
#pragma unroll
    for (int i = 0; i < 4; ++i) {
      const int yy = py[i] + dy, xx = px[i] + dx;
      ok[i] = (unsigned)yy < (unsigned)H && (unsigned)xx < (unsigned)H;
      const int ys = ok[i] ? (a.up ? yy >> 1 : yy) : 0;
      const int xs = ok[i] ? (a.up ? xx >> 1 : xx) : 0;
      src[i] = a.in.p + ((img[i] + (int64_t)ys * Hin + xs) * a.in.cs + a.in.co + 8 * q);
    }
    for (int c0 = 0; c0 < a.Cin; c0 += 32) {
      bf16x8 A[4], Bv[2];
#pragma unroll
      for (int i = 0; i < 4; ++i) A[i] = ok[i] ? ld8(src[i] + c0) : zero8();
#pragma unroll
      for (int j = 0; j < 2; ++j) Bv[j] = ld8(wrow[j] + tap * a.Cin + c0);
#pragma unroll
      for (int i = 0; i < 4; ++i)
#pragma unroll
        for (int j = 0; j < 2; ++j)
          acc[i][j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(A[i], Bv[j], acc[i][j], 0, 0, 0);
    }
  }

#pragma unroll
  for (int j = 0; j < 2; ++j) {
    const int co = cot * 32 + 16 * j + r;
    const float bias = a.bias ? a.bias[co] : 0.f;
#pragma unroll
    for (int i = 0; i < 4; ++i) {
#pragma unroll
      for (int e = 0; e < 4; ++e) {
        const int64_t P = pt * 64 + 16 * i + 4 * q + e;
        float v = acc[i][j][e] + bias;
        if (a.relu) v = fmaxf(v, 0.f);
        if (a.mask.p && !(bf2f(a.mask.p[P * a.mask.cs + a.mask.co + co]) > 0.f)) v = 0.f;
        a.out.p[P * a.out.cs + a.out.co + co] = f2bf(v);
      }
    }
  }
}

// LDS-tiled variant for grids of at least 32 x 32: a workgroup owns an
// output tile of TR rows x 32 columns x CO channels (TR = 2 NPT, CO = 16 NCT)
// and walks the input channels in chunks of 32.  Per chunk it stages the
// (TR + 2) x 34 input patch (all nine taps' pixels, zeros outside the grid,
// the nearest-neighbour upsampling applied on the way in) and the CO x 9 x 32
// weights in LDS with 16-byte loads; each wavefront then takes NPT/2 rows of
// the tile (NPT MFMA tiles of 16 pixels) x CO channels, reading its A and B
// operands from LDS: 16 consecutive pixels' 32 channels are one contiguous
// kilobyte (conflict-free), and the weight rows are padded so that 16 output
// channels' reads fall into distinct banks.
constexpr int kWS = 9 * 32 + 8;   // LDS row stride (bf16) of one output channel's weights

__device__ __forceinline__ bf16x8 lds8(const uint16_t* p) {
  return __builtin_bit_cast(bf16x8, *reinterpret_cast<const u32x4*>(p));
}

template <int NPT, int NCT>
__global__ __launch_bounds__(256, 2) void conv3x3_lds_kernel(ConvArgs a, int n_blocks) {
  constexpr int TR = 2 * NPT, TC = 32, CO = 16 * NCT;
  constexpr int PR = TR + 2, PC = TC + 2;
  __shared__ __align__(16) uint16_t patch[PR * PC * 32];
  __shared__ __align__(16) uint16_t wts[CO * kWS];
  const int64_t blk = xcd_block();
  if (blk >= n_blocks) return;
  const int H = a.H, Hin = a.up ? (H >> 1) : H;
  const int nco = a.Cout / CO, ntx = H / TC, nty = H / TR;
  // output-channel tiles fastest: consecutive blocks share the input patch
  const int cot = (int)(blk % nco);
  int64_t t = blk / nco;
  const int tx = (int)(t % ntx);
  t /= ntx;
  const int ty = (int)(t % nty);
  const int64_t n = t / nty;
  const int y0 = ty * TR, x0 = tx * TC;
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int r = lane & 15, q = lane >> 4;
  const int64_t img = n * Hin * Hin;

  f32x4 acc[NPT][NCT];
#pragma unroll
  for (int i = 0; i < NPT; ++i)
#pragma unroll
    for (int j = 0; j < NCT; ++j) acc[i][j] = f32x4{0.f, 0.f, 0.f, 0.f};

  for (int c0 = 0; c0 < a.Cin; c0 += 32) {
    __syncthreads();  // the previous chunk's reads are done
    for (int e = tid; e < PR * PC * 4; e += 256) {
      const int pix = e >> 2, g = e & 3;
      const int py = pix / PC, px = pix - py * PC;
      const int yy = y0 - 1 + py, xx = x0 - 1 + px;
      bf16x8 v = zero8();
      if ((unsigned)yy < (unsigned)H && (unsigned)xx < (unsigned)H) {
        const int ys = a.up ? yy >> 1 : yy, xs = a.up ? xx >> 1 : xx;
        v = ld8(a.in.p + ((img + (int64_t)ys * Hin + xs) * a.in.cs + a.in.co + c0 + 8 * g));
      }
      *reinterpret_cast<bf16x8*>(patch + pix * 32 + 8 * g) = v;
    }
    for (int e = tid; e < CO * 36; e += 256) {
      const int co = e / 36, rem = e - co * 36, tap = rem >> 2, g = rem & 3;
      *reinterpret_cast<bf16x8*>(wts + co * kWS + tap * 32 + 8 * g) =
          ld8(a.w + ((size_t)(cot * CO + co) * 9 + tap) * a.Cin + c0 + 8 * g);
    }
    __syncthreads();
#pragma unroll
    for (int tap = 0; tap < 9; ++tap) {
      const int dy = tap / 3, dx = tap % 3;   // patch offsets (the tap's -1 .. 1 plus the halo)
      bf16x8 Bv[NCT];
#pragma unroll
      for (int j = 0; j < NCT; ++j) Bv[j] = lds8(wts + (16 * j + r) * kWS + tap * 32 + 8 * q);
#pragma unroll
      for (int i = 0; i < NPT; ++i) {
        const int prow = wave * (NPT / 2) + (i >> 1) + dy, pcol = 16 * (i & 1) + r + dx;
        const bf16x8 A = lds8(patch + (prow * PC + pcol) * 32 + 8 * q);
#pragma unroll
        for (int j = 0; j < NCT; ++j)
          acc[i][j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(A, Bv[j], acc[i][j], 0, 0, 0);
      }
    }
  }

#pragma unroll
  for (int j = 0; j < NCT; ++j) {
    const int co = cot * CO + 16 * j + r;
    const float bias = a.bias ? a.bias[co] : 0.f;
#pragma unroll
    for (int i = 0; i < NPT; ++i) {
      const int y = y0 + wave * (NPT / 2) + (i >> 1);
#pragma unroll
      for (int e = 0; e < 4; ++e) {
        const int x = x0 + 16 * (i & 1) + 4 * q + e;
        const int64_t P = (n * H + y) * H + x;
        float v = acc[i][j][e] + bias;
        if (a.relu) v = fmaxf(v, 0.f);
        if (a.mask.p && !(bf2f(a.mask.p[P * a.mask.cs + a.mask.co + co]) > 0.f)) v = 0.f;
        a.out.p[P * a.out.cs + a.out.co + co] = f2bf(v);
      }
    }
  }
}

// -------------------------------------------------------- weight gradient
constexpr int kLD = 64 + 8;  // LDS row stride (bf16) of the staged chunks

template <int TCO, int TCI>
__global__ __launch_bounds__(64 * (TCO / 32) * (TCI / 32)) void wgrad_kernel(WgradArgs a,
                                                                          int n_chunks,
                                                                          int cps, int nci_t) {
  constexpr int NT = 64 * (TCO / 32) * (TCI / 32);
  __shared__ __attribute__((aligned(16))) uint16_t sz[TCO * kLD];
  __shared__ __attribute__((aligned(16))) uint16_t sx[TCI * kLD];
  const int split = blockIdx.x, tap = blockIdx.y;
  const int cot = blockIdx.z / nci_t, cit = blockIdx.z % nci_t;
  const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
  const int wco = (w / (TCI / 32)) * 32, wci = (w % (TCI / 32)) * 32;
  const int r = lane & 15, q = lane >> 4;
  const int dy = tap / 3 - 1, dx = tap % 3 - 1;
  const int H = a.H, HW = H * H;
  const int Hin = a.up ? (H >> 1) : H;
  const bool do_bias = tap == 4 && cit == 0;

  f32x4 acc[2][2];
#pragma unroll
  for (int i = 0; i < 2; ++i)
#pragma unroll
    for (int j = 0; j < 2; ++j) acc[i][j] = f32x4{0.f, 0.f, 0.f, 0.f};
  float bsum = 0.f;

  const int c_begin = split * cps, c_end = min(n_chunks, c_begin + cps);
  for (int ch = c_begin; ch < c_end; ++ch) {
    const int64_t P0 = (int64_t)ch * 64;
    for (int e = tid; e < 64 * (TCO / 8); e += NT) {
      const int p = e / (TCO / 8), cg = e % (TCO / 8);
      const u32x4 v = *reinterpret_cast<const u32x4*>(a.dz.p + (P0 + p) * a.dz.cs + a.dz.co +
                                                      cot * TCO + cg * 8);
#pragma unroll
      for (int j = 0; j < 8; ++j) sz[(cg * 8 + j) * kLD + p] = (uint16_t)(v[j >> 1] >> (16 * (j & 1)));
    }
    for (int e = tid; e < 64 * (TCI / 8); e += NT) {
      const int p = e / (TCI / 8), cg = e % (TCI / 8);
      const int64_t P = P0 + p;
      const int64_t n = P / HW;
      const int rem = (int)(P - n * HW);
      const int yy = rem / H + dy, xx = rem % H + dx;
      u32x4 v = {0u, 0u, 0u, 0u};
      if ((unsigned)yy < (unsigned)H && (unsigned)xx < (unsigned)H) {
        const int ys = a.up ? yy >> 1 : yy, xs = a.up ? xx >> 1 : xx;
        v = *reinterpret_cast<const u32x4*>(a.in.p + ((n * Hin + ys) * Hin + xs) * a.in.cs +
                                            a.in.co + cit * TCI + cg * 8);
      }
#pragma unroll
      for (int j = 0; j < 8; ++j) sx[(cg * 8 + j) * kLD + p] = (uint16_t)(v[j >> 1] >> (16 * (j & 1)));
    }
    __syncthreads();
    if (do_bias && tid < TCO)
      for (int p = 0; p < 64; ++p) bsum += bf2f(sz[tid * kLD + p]);
#pragma unroll
    for (int ks = 0; ks < 2; ++ks) {
      bf16x8 A[2], Bv[2];
#pragma unroll
      for (int i = 0; i < 2; ++i) A[i] = ld8(sz + (wco + 16 * i + r) * kLD + 32 * ks + 8 * q);
#pragma unroll
      for (int j = 0; j < 2; ++j) Bv[j] = ld8(sx + (wci + 16 * j + r) * kLD + 32 * ks + 8 * q);
#pragma unroll
      for (int i = 0; i < 2; ++i)
#pragma unroll
        for (int j = 0; j < 2; ++j)
          acc[i][j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(A[i], Bv[j], acc[i][j], 0, 0, 0);
    }
    __syncthreads();
  }

  const size_t nw = (size_t)a.Cout * 9 * a.Cin;
  float* wp = a.part + (size_t)split * nw;
#pragma unroll
  for (int i = 0; i < 2; ++i)
#pragma unroll
    for (int j = 0; j < 2; ++j)
#pragma unroll
      for (int e = 0; e < 4; ++e) {
        const int co = cot * TCO + wco + 16 * i + 4 * q + e;
        const int ci = cit * TCI + wci + 16 * j + r;
        wp[((size_t)co * 9 + tap) * a.Cin + ci] = acc[i][j][e];
      }
  if (do_bias && tid < TCO)
    a.part[(size_t)gridDim.x * nw + (size_t)split * a.Cout + cot * TCO + tid] = bsum;
}

// Weight gradient on grids of at least 64 columns (a multiple of 64): the
// pixels are walked in 64-pixel row segments and a workgroup forms all nine
// taps of its TCO x TCI tile, so each segment's dz (TCO channels x 64
// pixels) and the three input rows the taps reach (TCI channels x 66 pixels,
// zeros outside the grid) are staged once, transposed to pixel-contiguous
// rows.  A tap's row offset selects the staged row and its column offset is
// applied when the B operand is read (an aligned 16-byte read, the next four
// bytes and a byte alignment).  The (TCO/32) x (TCI/32) blocks of 32 x 32
// go to the wavefronts, a block's nine taps dealt out among its wavefronts.
constexpr int kLX = 80;   // LDS row stride (bf16) of the staged input rows (66 pixels + pad)

__device__ __forceinline__ bf16x8 lds8_at(const uint16_t* row, int s, int d) {
  // row[s .. s+7] with s = 8 m + d, d in {0, 1, 2}
  const u32x4 lo = *reinterpret_cast<const u32x4*>(row + (s - d));
  if (d == 0) return __builtin_bit_cast(bf16x8, lo);
  const uint32_t hi = *reinterpret_cast<const uint32_t*>(row + (s - d) + 8);
  u32x4 o;
  if (d == 2) {
    o[0] = lo[1];
    o[1] = lo[2];
    o[2] = lo[3];
    o[3] = hi;
  } else {
    o[0] = __builtin_amdgcn_alignbyte(lo[1], lo[0], 2);
    o[1] = __builtin_amdgcn_alignbyte(lo[2], lo[1], 2);
    o[2] = __builtin_amdgcn_alignbyte(lo[3], lo[2], 2);
    o[3] = __builtin_amdgcn_alignbyte(hi, lo[3], 2);
  }
  return __builtin_bit_cast(bf16x8, o);
}

template <int TCO, int TCI>
__global__ __launch_bounds__(256) void wgrad_row_kernel(WgradArgs a, int n_chunks, int cps,
                                                        int nci_t) {
  constexpr int NB = (TCO / 32) * (TCI / 32);   // 32 x 32 blocks of the tile
  constexpr int WPB = 4 / NB;                   // wavefronts per block
  constexpr int NTW = (9 + WPB - 1) / WPB;      // taps per wavefront, at most
  __shared__ __attribute__((aligned(16))) uint16_t sz[TCO * kLD];
  __shared__ __attribute__((aligned(16))) uint16_t sx[3 * TCI * kLX];
  const int split = blockIdx.x;
  const int cot = blockIdx.z / nci_t, cit = blockIdx.z % nci_t;
  const int tid = threadIdx.x, lane = tid & 63;
  const int w = __builtin_amdgcn_readfirstlane(tid >> 6);
  const int blk = w / WPB, wib = w % WPB;
  const int wco = (blk / (TCI / 32)) * 32, wci = (blk % (TCI / 32)) * 32;
  const int r = lane & 15, q = lane >> 4;
  const int H = a.H, Hin = a.up ? (H >> 1) : H;
  const int spr = H / 64;   // segments per row
  const bool do_bias = cit == 0;

  f32x4 acc[NTW][2][2];
#pragma unroll
  for (int it = 0; it < NTW; ++it)
#pragma unroll
    for (int i = 0; i < 2; ++i)
#pragma unroll
      for (int j = 0; j < 2; ++j) acc[it][i][j] = f32x4{0.f, 0.f, 0.f, 0.f};
  float bsum = 0.f;

  const int c_begin = split * cps, c_end = min(n_chunks, c_begin + cps);
  for (int ch = c_begin; ch < c_end; ++ch) {
    const int64_t grow = ch / spr;                 // n H + y
    const int x0 = (int)(ch - grow * spr) * 64;
    const int64_t n = grow / H;
    const int y = (int)(grow - n * H);
    const int64_t P0 = grow * H + x0;
    for (int e = tid; e < 64 * (TCO / 8); e += 256) {
      const int p = e / (TCO / 8), cg = e % (TCO / 8);
      const u32x4 v = *reinterpret_cast<const u32x4*>(a.dz.p + (P0 + p) * a.dz.cs + a.dz.co +
                                                      cot * TCO + cg * 8);
#pragma unroll
      for (int j = 0; j < 8; ++j) sz[(cg * 8 + j) * kLD + p] = (uint16_t)(v[j >> 1] >> (16 * (j & 1)));
    }
    for (int e = tid; e < 3 * 66 * (TCI / 8); e += 256) {
      const int cg = e % (TCI / 8), rest = e / (TCI / 8);
      const int j = rest % 66, dy = rest / 66;
      const int yy = y + dy - 1, xx = x0 + j - 1;
      u32x4 v = {0u, 0u, 0u, 0u};
      if ((unsigned)yy < (unsigned)H && (unsigned)xx < (unsigned)H) {
        const int ys = a.up ? yy >> 1 : yy, xs = a.up ? xx >> 1 : xx;
        v = *reinterpret_cast<const u32x4*>(a.in.p + ((n * Hin + ys) * Hin + xs) * a.in.cs +
                                            a.in.co + cit * TCI + cg * 8);
      }
#pragma unroll
      for (int jj = 0; jj < 8; ++jj)
        sx[(dy * TCI + cg * 8 + jj) * kLX + j] = (uint16_t)(v[jj >> 1] >> (16 * (jj & 1)));
    }
    __syncthreads();
    if (do_bias && tid < TCO)
      for (int p = 0; p < 64; ++p) bsum += bf2f(sz[tid * kLD + p]);
#pragma unroll
    for (int ks = 0; ks < 2; ++ks) {
      bf16x8 A[2];
#pragma unroll
      for (int i = 0; i < 2; ++i) A[i] = ld8(sz + (wco + 16 * i + r) * kLD + 32 * ks + 8 * q);
#pragma unroll
      for (int it = 0; it < NTW; ++it) {
        const int t = wib + it * WPB;
        if (t < 9) {   // uniform over the wavefront
          const int dy = t / 3, dx = t % 3;
          bf16x8 Bv[2];
#pragma unroll
          for (int j = 0; j < 2; ++j)
            Bv[j] = lds8_at(sx + (dy * TCI + wci + 16 * j + r) * kLX, 32 * ks + 8 * q + dx, dx);
#pragma unroll
          for (int i = 0; i < 2; ++i)
#pragma unroll
            for (int j = 0; j < 2; ++j)
              acc[it][i][j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(A[i], Bv[j], acc[it][i][j], 0, 0, 0);
        }
      }
    }
    __syncthreads();
  }

  const size_t nw = (size_t)a.Cout * 9 * a.Cin;
  float* wp = a.part + (size_t)split * nw;
#pragma unroll
  for (int it = 0; it < NTW; ++it) {
    const int t = wib + it * WPB;
    if (t < 9) {
#pragma unroll
      for (int i = 0; i < 2; ++i)
#pragma unroll
        for (int j = 0; j < 2; ++j)
#pragma unroll
          for (int e = 0; e < 4; ++e) {
            const int co = cot * TCO + wco + 16 * i + 4 * q + e;
            const int ci = cit * TCI + wci + 16 * j + r;
            wp[((size_t)co * 9 + t) * a.Cin + ci] = acc[it][i][j][e];
          }
    }
  }
  if (do_bias && tid < TCO)
    a.part[(size_t)gridDim.x * nw + (size_t)split * a.Cout + cot * TCO + tid] = bsum;
}

// dw[i] = sum_s part[s][i], db[c] = sum_s bpart[s][c]: a workgroup takes 64
// entries, its four wavefronts the splits s = 4 m + w (each summed in
// order), combined in the order w = 0 .. 3 (a fixed order throughout).
__global__ __launch_bounds__(256) void wgrad_reduce_kernel(const float* part, int nsplit,
                                                           int64_t nw, int Cout, float* dw,
                                                           float* db) {
  __shared__ float red[4][64];
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  const int64_t i = (int64_t)blockIdx.x * 64 + lane;
  float s = 0.f;
  if (i < nw) {
#pragma unroll 4
    for (int k = w; k < nsplit; k += 4) s += part[(size_t)k * nw + i];
  } else if (i < nw + Cout) {
    const float* bp = part + (size_t)nsplit * nw;
    const int c = (int)(i - nw);
#pragma unroll 4
    for (int k = w; k < nsplit; k += 4) s += bp[(size_t)k * Cout + c];
  }
  red[w][lane] = s;
  __syncthreads();
  if (w == 0) {
    const float t = (red[0][lane] + red[1][lane]) + (red[2][lane] + red[3][lane]);
    if (i < nw)
      dw[i] = t;
    else if (i < nw + Cout)
      db[i - nw] = t;
  }
}

struct WgradPlan {
  int tco, tci, nco_t, nci_t, n_chunks, cps, nsplit;
};

// rows: the row-segment kernel (grids of 64 columns or more, all nine taps
// per workgroup, about 512 workgroups), else the per-tap kernel (about 2048)
static bool wgrad_rows(int H) { return H >= 64 && H % 64 == 0; }

WgradPlan wgrad_plan(int Cout, int Cin, int B, int H) {
  WgradPlan p;
  p.tco = Cout >= 64 ? 64 : 32;
  p.tci = Cin >= 64 ? 64 : 32;
  p.nco_t = Cout / p.tco;
  p.nci_t = Cin / p.tci;
  p.n_chunks = (int)((int64_t)B * H * H / 64);
  const int base = (wgrad_rows(H) ? 1 : 9) * p.nco_t * p.nci_t;
  const int target = wgrad_rows(H) ? 512 : 2048;
  int want = (target + base - 1) / base;
  want = std::max(1, std::min(want, p.n_chunks));
  p.cps = (p.n_chunks + want - 1) / want;
  p.nsplit = (p.n_chunks + p.cps - 1) / p.cps;
  return p;
}

// ------------------------------------------------------------ first layer
// First layer (one input channel): a lane per pixel computes all Cout
// channels (weights and biases in LDS as float) and stores them eight at a
// time (16 bytes); each channel's sum runs over the taps in order, as the
// definition writes it (taps outside the grid add zero).
__global__ __launch_bounds__(256) void conv_in_kernel(const float* u, float in_scale,
                                                      const uint16_t* w, const float* bias,
                                                      Tensor out, int Cout, int B, int H) {
  extern __shared__ float wsh[];   // [Cout][9] weights, then [Cout] biases
  for (int e = threadIdx.x; e < Cout * 10; e += 256)
    wsh[e] = e < Cout * 9 ? bf2f(w[e]) : bias[e - Cout * 9];
  __syncthreads();
  const int64_t P = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (P >= (int64_t)B * H * H) return;
  const int64_t n = P / (H * H);
  const int rem = (int)(P - n * H * H);
  const int y = rem / H, x = rem - (rem / H) * H;
  const float* un = u + n * H * H;
  float uv[9];
#pragma unroll
  for (int tap = 0; tap < 9; ++tap) {
    const int yy = y + tap / 3 - 1, xx = x + tap % 3 - 1;
    uv[tap] = ((unsigned)yy < (unsigned)H && (unsigned)xx < (unsigned)H)
                  ? in_scale * un[yy * H + xx] : 0.f;
  }
  uint16_t* dst = out.p + P * out.cs + out.co;
  for (int c0 = 0; c0 < Cout; c0 += 8) {
    u32x4 pk;
#pragma unroll
    for (int k = 0; k < 8; k += 2) {
      float z[2];
#pragma unroll
      for (int h = 0; h < 2; ++h) {
        const float* wc = wsh + (c0 + k + h) * 9;
        float acc = 0.f;
#pragma unroll
        for (int tap = 0; tap < 9; ++tap) acc += wc[tap] * uv[tap];
        z[h] = fmaxf(acc + wsh[Cout * 9 + c0 + k + h], 0.f);
      }
      pk[k >> 1] = (uint32_t)f2bf(z[0]) | ((uint32_t)f2bf(z[1]) << 16);
    }
    *reinterpret_cast<u32x4*>(dst + c0) = pk;
  }
}

// entry t = k * Cout + co: tap k < 9 (weight) or k = 9 (bias) of channel co,
// summed over this workgroup's pixels [p0, p1).  Per chunk of 32 channels a
// lane takes one group of 8 channels (tid & 3) of every 64th pixel (pixel
// lane tid >> 2), with 16-byte loads of dz, and sums its 80 products in
// order; the 64 pixel lanes are then added by a butterfly within each
// wavefront and the four wavefronts in order (fixed order throughout).
__global__ __launch_bounds__(256) void wgrad_in_kernel(const uint16_t* dz, int Cout,
                                                       const float* u, float in_scale, int B,
                                                       int H, int64_t cps, float* part) {
  __shared__ float red[4][4][80];
  const int64_t npx = (int64_t)B * H * H;
  const int64_t p0 = (int64_t)blockIdx.x * cps, p1 = min(npx, p0 + cps);
  const int tid = threadIdx.x, cg = tid & 3, pl = tid >> 2, w = tid >> 6;
  const int HH = H * H;
  for (int c0 = 0; c0 < Cout; c0 += 32) {
    float acc[10][8];
#pragma unroll
    for (int k = 0; k < 10; ++k)
#pragma unroll
      for (int j = 0; j < 8; ++j) acc[k][j] = 0.f;
    for (int64_t P = p0 + pl; P < p1; P += 64) {
      const int64_t n = P / HH;
      const int rem = (int)(P - n * HH);
      const int y = rem / H, x = rem - (rem / H) * H;
      const float* un = u + n * HH;
      const u32x4 gv = *reinterpret_cast<const u32x4*>(dz + P * Cout + c0 + 8 * cg);
      float g[8];
#pragma unroll
      for (int j = 0; j < 8; ++j) g[j] = bf2f((uint16_t)(gv[j >> 1] >> (16 * (j & 1))));
#pragma unroll
      for (int k = 0; k < 9; ++k) {
        const int yy = y + k / 3 - 1, xx = x + k % 3 - 1;
        const float uv = ((unsigned)yy < (unsigned)H && (unsigned)xx < (unsigned)H)
                             ? in_scale * un[yy * H + xx] : 0.f;
#pragma unroll
        for (int j = 0; j < 8; ++j) acc[k][j] = fmaf(g[j], uv, acc[k][j]);
      }
#pragma unroll
      for (int j = 0; j < 8; ++j) acc[9][j] += g[j];
    }
    // the 16 pixel lanes of a wavefront with the same channel group: lanes
    // 4 apart, added by a butterfly over lane bits 2..5
#pragma unroll
    for (int k = 0; k < 10; ++k)
#pragma unroll
      for (int j = 0; j < 8; ++j) {
        float v = acc[k][j];
        for (int o = 4; o < 64; o <<= 1) v += __shfl_xor(v, o, 64);
        acc[k][j] = v;
      }
    if ((tid & 63) < 4) {
#pragma unroll
      for (int k = 0; k < 10; ++k)
#pragma unroll
        for (int j = 0; j < 8; ++j) red[w][cg][k * 8 + j] = acc[k][j];
    }
    __syncthreads();
    for (int e = tid; e < 320; e += 256) {
      const int g4 = e / 80, kj = e % 80, k = kj / 8, j = kj % 8;
      const float v = (red[0][g4][kj] + red[1][g4][kj]) + (red[2][g4][kj] + red[3][g4][kj]);
      part[(size_t)blockIdx.x * 10 * Cout + k * Cout + c0 + 8 * g4 + j] = v;
    }
    __syncthreads();
  }
}

// dw, db of the first layer: a workgroup takes 16 entries t, its lanes
// (t, g) the splits g, g + 16, ... (each in order), combined over g in order.
__global__ __launch_bounds__(256) void wgrad_in_reduce_kernel(const float* part, int nsplit,
                                                              int Cout, float* dw, float* db) {
  __shared__ float red[16][17];
  const int e = threadIdx.x & 15, g = threadIdx.x >> 4;
  const int t = blockIdx.x * 16 + e;
  float s = 0.f;
  if (t < 10 * Cout) {
#pragma unroll 4
    for (int k = g; k < nsplit; k += 16) s += part[(size_t)k * 10 * Cout + t];
  }
  red[g][e] = s;
  __syncthreads();
  if (g == 0 && t < 10 * Cout) {
    float v = 0.f;
#pragma unroll
    for (int h = 0; h < 16; ++h) v += red[h][e];
    const int co = t % Cout, k = t / Cout;
    if (k < 9)
      dw[co * 9 + k] = v;
    else
      db[co] = v;
  }
}

// ------------------------------------------------------- pool / up / head
// The pooling and upsampling kernels take a lane per (pixel, group of 8
// channels): 16-byte loads and stores of NHWC rows (C a multiple of 8).
__device__ __forceinline__ float lane8(const u32x4& v, int k) {
  return bf2f((uint16_t)(v[k >> 1] >> (16 * (k & 1))));
}
__device__ __forceinline__ u32x4 ld16(const uint16_t* p) { return *reinterpret_cast<const u32x4*>(p); }

__global__ void pool_kernel(Tensor in, Tensor out, int C, int B, int H) {
  const int Ho = H >> 1, G = C >> 3;
  const int64_t idx = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (idx >= (int64_t)B * Ho * Ho * G) return;
  const int64_t Q = idx / G;
  const int c = 8 * (int)(idx - Q * G);
  const int64_t n = Q / (Ho * Ho);
  const int rem = (int)(Q - n * Ho * Ho);
  const int y = 2 * (rem / Ho), x = 2 * (rem % Ho);
  const int64_t P = (n * H + y) * H + x;
  const uint16_t* s = in.p + in.co + c;
  const u32x4 a = ld16(s + P * in.cs), b = ld16(s + (P + 1) * in.cs);
  const u32x4 d = ld16(s + (P + H) * in.cs), e = ld16(s + (P + H + 1) * in.cs);
  u32x4 o;
#pragma unroll
  for (int k = 0; k < 8; k += 2) {
    const float v0 = lane8(a, k) + lane8(b, k) + lane8(d, k) + lane8(e, k);
    const float v1 = lane8(a, k + 1) + lane8(b, k + 1) + lane8(d, k + 1) + lane8(e, k + 1);
    o[k >> 1] = (uint32_t)f2bf(0.25f * v0) | ((uint32_t)f2bf(0.25f * v1) << 16);
  }
  *reinterpret_cast<u32x4*>(out.p + Q * out.cs + out.co + c) = o;
}

__global__ void pool_back_add_kernel(Tensor dp, Tensor e, Tensor de, int C, int B, int H) {
  const int G = C >> 3;
  const int64_t idx = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (idx >= (int64_t)B * H * H * G) return;
  const int64_t P = idx / G;
  const int c = 8 * (int)(idx - P * G);
  const int64_t n = P / (H * H);
  const int rem = (int)(P - n * H * H);
  const int Ho = H >> 1;
  const int64_t Q = (n * Ho + (rem / H) / 2) * Ho + (rem % H) / 2;
  uint16_t* d = de.p + P * de.cs + de.co + c;
  const u32x4 dv = ld16(d), pv = ld16(dp.p + Q * dp.cs + dp.co + c);
  const u32x4 ev = ld16(e.p + P * e.cs + e.co + c);
  u32x4 o;
#pragma unroll
  for (int k = 0; k < 8; k += 2) {
    float v[2];
#pragma unroll
    for (int h = 0; h < 2; ++h) {
      v[h] = lane8(dv, k + h) + 0.25f * lane8(pv, k + h);
      if (!(lane8(ev, k + h) > 0.f)) v[h] = 0.f;
    }
    o[k >> 1] = (uint32_t)f2bf(v[0]) | ((uint32_t)f2bf(v[1]) << 16);
  }
  *reinterpret_cast<u32x4*>(d) = o;
}

__global__ void up_back_kernel(Tensor du, Tensor d, Tensor dd, int C, int B, int H) {
  const int G = C >> 3;
  const int64_t idx = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (idx >= (int64_t)B * H * H * G) return;
  const int64_t Q = idx / G;
  const int c = 8 * (int)(idx - Q * G);
  const int64_t n = Q / (H * H);
  const int rem = (int)(Q - n * H * H);
  const int H2 = 2 * H;
  const int64_t P = (n * H2 + 2 * (rem / H)) * H2 + 2 * (rem % H);
  const uint16_t* s = du.p + du.co + c;
  const u32x4 a = ld16(s + P * du.cs), b = ld16(s + (P + 1) * du.cs);
  const u32x4 e = ld16(s + (P + H2) * du.cs), f = ld16(s + (P + H2 + 1) * du.cs);
  const u32x4 m = ld16(d.p + Q * d.cs + d.co + c);
  u32x4 o;
#pragma unroll
  for (int k = 0; k < 8; k += 2) {
    float v[2];
#pragma unroll
    for (int h = 0; h < 2; ++h) {
      v[h] = lane8(a, k + h) + lane8(b, k + h) + lane8(e, k + h) + lane8(f, k + h);
      if (!(lane8(m, k + h) > 0.f)) v[h] = 0.f;
    }
    o[k >> 1] = (uint32_t)f2bf(v[0]) | ((uint32_t)f2bf(v[1]) << 16);
  }
  *reinterpret_cast<u32x4*>(dd.p + Q * dd.cs + dd.co + c) = o;
}

__global__ void head_kernel(Tensor d, int C, const float* head, const float* u, float in_scale,
                            float* x0, int64_t npx) {
  const int64_t P = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (P >= npx) return;
  const uint16_t* dp = d.p + P * d.cs + d.co;
  float s = 0.f;
  for (int c = 0; c < C; c += 8) {   // 16-byte loads, channels summed in order
    const u32x4 v = ld16(dp + c);
#pragma unroll
    for (int k = 0; k < 8; ++k) s += head[c + k] * lane8(v, k);
  }
  x0[P] = s + head[C] + head[C + 1] * (in_scale * u[P]);
}

// per workgroup: sums of dx0 * D[c] (c < C), dx0, dx0 * uh and diff^2 (in
// that order), each reduced within a wavefront by shuffles and across the
// four wavefronts in a fixed order
__device__ __forceinline__ double wave_sum64(double v) {
  for (int o = 32; o > 0; o >>= 1) v += __shfl_down(v, o, 64);
  return v;
}

__global__ __launch_bounds__(256) void head_back_kernel(Tensor d, int C, const float* head,
                                                        const float* u, float in_scale,
                                                        const float* x0, const float* target,
                                                        int64_t npx, Tensor dz, double* part) {
  // Per lane: every (gridDim.x * 256)-th pixel from its own, each quantity
  // summed over them in order; then across the wavefront by shuffles and
  // across the four wavefronts in order.  Channels go eight at a time
  // (16-byte loads of D and stores of dz).
  extern __shared__ double red[];  // [4][C + 3]
  const int w = threadIdx.x >> 6, lane = threadIdx.x & 63;
  const int64_t P0 = (int64_t)blockIdx.x * 256 + threadIdx.x;
  const int64_t step = (int64_t)gridDim.x * 256;
  const float inv = 2.f / (float)npx;
  for (int c0 = 0; c0 < C; c0 += 8) {
    double acc[8];
#pragma unroll
    for (int j = 0; j < 8; ++j) acc[j] = 0.0;
    for (int64_t P = P0; P < npx; P += step) {
      const float g = inv * (x0[P] - target[P]);
      const u32x4 dv = *reinterpret_cast<const u32x4*>(d.p + P * d.cs + d.co + c0);
      u32x4 o;
#pragma unroll
      for (int j = 0; j < 8; j += 2) {
        const float a = lane8(dv, j), b = lane8(dv, j + 1);
        acc[j] += (double)g * a;
        acc[j + 1] += (double)g * b;
        o[j >> 1] = (uint32_t)f2bf(a > 0.f ? g * head[c0 + j] : 0.f) |
                    ((uint32_t)f2bf(b > 0.f ? g * head[c0 + j + 1] : 0.f) << 16);
      }
      *reinterpret_cast<u32x4*>(dz.p + P * dz.cs + dz.co + c0) = o;
    }
#pragma unroll
    for (int j = 0; j < 8; ++j) {
      const double v = wave_sum64(acc[j]);
      if (lane == 0) red[w * (C + 3) + c0 + j] = v;
    }
  }
  double a1 = 0.0, a2 = 0.0, a3 = 0.0;
  for (int64_t P = P0; P < npx; P += step) {
    const float diff = x0[P] - target[P];
    const float g = inv * diff;
    a1 += g;
    a2 += (double)g * (in_scale * u[P]);
    a3 += (double)diff * diff;
  }
  a1 = wave_sum64(a1);
  a2 = wave_sum64(a2);
  a3 = wave_sum64(a3);
  if (lane == 0) {
    red[w * (C + 3) + C] = a1;
    red[w * (C + 3) + C + 1] = a2;
    red[w * (C + 3) + C + 2] = a3;
  }
  __syncthreads();
  for (int k = threadIdx.x; k < C + 3; k += 256)
    part[(size_t)blockIdx.x * (C + 3) + k] =
        (red[k] + red[(C + 3) + k]) + (red[2 * (C + 3) + k] + red[3 * (C + 3) + k]);
}

// out[k] = sum over workgroups of part[wg][k]: one workgroup per quantity,
// strided partial sums and a tree, both in a fixed order
__global__ __launch_bounds__(256) void head_reduce_kernel(const double* part, int nblk, int C,
                                                          double* loss, float* dhead,
                                                          double inv_npx) {
  __shared__ double red[256];
  const int k = blockIdx.x;
  double s = 0.0;
  for (int b = threadIdx.x; b < nblk; b += 256) s += part[(size_t)b * (C + 3) + k];
  red[threadIdx.x] = s;
  __syncthreads();
  for (int o = 128; o > 0; o >>= 1) {
    if ((int)threadIdx.x < o) red[threadIdx.x] += red[threadIdx.x + o];
    __syncthreads();
  }
  if (threadIdx.x == 0) {
    if (k < C + 2)
      dhead[k] = (float)red[0];
    else
      *loss = red[0] * inv_npx;
  }
}

__global__ void adam_kernel(float* p, const float* g, float* m, float* v, int64_t n, float b1,
                            float b2, float lr_t, float eps_t) {
  const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (i >= n) return;
  const float gi = g[i];
  const float mi = b1 * m[i] + (1.f - b1) * gi;
  const float vi = b2 * v[i] + (1.f - b2) * gi * gi;
  m[i] = mi;
  v[i] = vi;
  p[i] -= lr_t * mi / (sqrtf(vi) + eps_t);
}

__global__ void cast_weights_kernel(const float* w, uint16_t* w16, uint16_t* wt16, int Cout,
                                    int Cin) {
  const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (i >= (int64_t)Cout * 9 * Cin) return;
  const int co = (int)(i / (9 * Cin));
  const int rem = (int)(i - (int64_t)co * 9 * Cin);
  const int tap = rem / Cin, ci = rem % Cin;
  const uint16_t h = f2bf(w[i]);
  w16[i] = h;
  if (wt16) wt16[((size_t)ci * 9 + (8 - tap)) * Cout + co] = h;
}

__global__ void zero_kernel(float* x, int64_t n) {
  const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (i < n) x[i] = 0.f;
}

unsigned blocks256(int64_t n) { return (unsigned)((n + 255) / 256); }

}  // namespace

// ----------------------------------------------------------------- launchers
hipError_t launch_conv3x3(const ConvArgs& a, hipStream_t st) {
  if (a.H >= 32 && a.H % 32 == 0 && a.Cin % 32 == 0) {
    if (a.Cout == 32) {   // 8 x 32 pixels x 32 channels per workgroup
      const int64_t blocks = (int64_t)a.B * (a.H / 8) * (a.H / 32);
      hipLaunchKernelGGL((conv3x3_lds_kernel<4, 2>), dim3(grid8(blocks)), dim3(256), 0, st, a,
                         (int)blocks);
      return hipGetLastError();
    }
    if (a.Cout % 64 == 0) {   // 8 x 32 pixels x 64 channels per workgroup
      const int64_t blocks = (int64_t)a.B * (a.H / 8) * (a.H / 32) * (a.Cout / 64);
      hipLaunchKernelGGL((conv3x3_lds_kernel<4, 4>), dim3(grid8(blocks)), dim3(256), 0, st, a,
                         (int)blocks);
      return hipGetLastError();
    }
  }
  const int64_t npx = (int64_t)a.B * a.H * a.H;
  const int64_t tiles = (npx / 64) * (a.Cout / 32);
  const int64_t blocks = (tiles + kCW - 1) / kCW;
  hipLaunchKernelGGL(conv3x3_kernel, dim3(grid8(blocks)), dim3(64 * kCW), 0, st, a, tiles);
  return hipGetLastError();
}

// Upper bound over every batch size up to B: a plan never uses more splits
// than min(ceil(2048 / base), n_chunks), and that bound grows with B.
size_t wgrad_part_floats(int Cout, int Cin, int B, int H) {
  const WgradPlan p = wgrad_plan(Cout, Cin, B, H);
  const int base = (wgrad_rows(H) ? 1 : 9) * p.nco_t * p.nci_t;
  const int target = wgrad_rows(H) ? 512 : 2048;
  const int bound = std::max(1, std::min((target + base - 1) / base, p.n_chunks));
  return (size_t)bound * ((size_t)Cout * 9 * Cin + Cout);
}

hipError_t launch_wgrad(const WgradArgs& a, hipStream_t st) {
  const WgradPlan p = wgrad_plan(a.Cout, a.Cin, a.B, a.H);
  if (wgrad_rows(a.H)) {
    const dim3 grid(p.nsplit, 1, p.nco_t * p.nci_t);
    if (p.tco == 64 && p.tci == 64)
      hipLaunchKernelGGL((wgrad_row_kernel<64, 64>), grid, dim3(256), 0, st, a, p.n_chunks, p.cps, p.nci_t);
    else if (p.tco == 64)
      hipLaunchKernelGGL((wgrad_row_kernel<64, 32>), grid, dim3(256), 0, st, a, p.n_chunks, p.cps, p.nci_t);
    else if (p.tci == 64)
      hipLaunchKernelGGL((wgrad_row_kernel<32, 64>), grid, dim3(256), 0, st, a, p.n_chunks, p.cps, p.nci_t);
    else
      hipLaunchKernelGGL((wgrad_row_kernel<32, 32>), grid, dim3(256), 0, st, a, p.n_chunks, p.cps, p.nci_t);
  } else {
  const dim3 grid(p.nsplit, 9, p.nco_t * p.nci_t);
  if (p.tco == 64 && p.tci == 64)
    hipLaunchKernelGGL((wgrad_kernel<64, 64>), grid, dim3(256), 0, st, a, p.n_chunks, p.cps, p.nci_t);
  else if (p.tco == 64)
    hipLaunchKernelGGL((wgrad_kernel<64, 32>), grid, dim3(128), 0, st, a, p.n_chunks, p.cps, p.nci_t);
  else if (p.tci == 64)
    hipLaunchKernelGGL((wgrad_kernel<32, 64>), grid, dim3(128), 0, st, a, p.n_chunks, p.cps, p.nci_t);
  else
    hipLaunchKernelGGL((wgrad_kernel<32, 32>), grid, dim3(64), 0, st, a, p.n_chunks, p.cps, p.nci_t);
  }
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  const int64_t nw = (int64_t)a.Cout * 9 * a.Cin;
  hipLaunchKernelGGL(wgrad_reduce_kernel, dim3((unsigned)((nw + a.Cout + 63) / 64)), dim3(256), 0,
                     st, (const float*)a.part, p.nsplit, nw, a.Cout, a.dw, a.db);
  return hipGetLastError();
}

hipError_t launch_conv_in(const float* u, double in_scale, const uint16_t* w, const float* bias,
                          Tensor out, int Cout, int B, int H, hipStream_t st) {
  const int64_t n = (int64_t)B * H * H;
  hipLaunchKernelGGL(conv_in_kernel, dim3(blocks256(n)), dim3(256), sizeof(float) * 10 * Cout, st,
                     u, (float)in_scale, w, bias, out, Cout, B, H);
  return hipGetLastError();
}

static int wgrad_in_splits(int B, int H) {
  const int64_t npx = (int64_t)B * H * H;
  return (int)std::min<int64_t>(512, std::max<int64_t>(1, npx / 1024));
}

size_t wgrad_in_part_floats(int Cout, int B, int H) {
  return (size_t)wgrad_in_splits(B, H) * 10 * Cout;
}

hipError_t launch_wgrad_in(const uint16_t* dz, int Cout, const float* u, double in_scale, int B,
                           int H, float* dw, float* db, float* part, hipStream_t st) {
  const int64_t npx = (int64_t)B * H * H;
  const int ns = wgrad_in_splits(B, H);
  const int64_t cps = (npx + ns - 1) / ns;
  hipLaunchKernelGGL(wgrad_in_kernel, dim3(ns), dim3(256), 0, st, dz, Cout, u, (float)in_scale,
                     B, H, cps, part);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(wgrad_in_reduce_kernel, dim3((unsigned)((10 * Cout + 15) / 16)), dim3(256), 0,
                     st, (const float*)part, ns, Cout, dw, db);
  return hipGetLastError();
}

hipError_t launch_pool(Tensor in, Tensor out, int C, int B, int H, hipStream_t st) {
  const int64_t n = (int64_t)B * (H / 2) * (H / 2) * (C / 8);
  hipLaunchKernelGGL(pool_kernel, dim3(blocks256(n)), dim3(256), 0, st, in, out, C, B, H);
  return hipGetLastError();
}

hipError_t launch_pool_back_add(Tensor dp, Tensor e, Tensor de, int C, int B, int H,
                                hipStream_t st) {
  const int64_t n = (int64_t)B * H * H * (C / 8);
  hipLaunchKernelGGL(pool_back_add_kernel, dim3(blocks256(n)), dim3(256), 0, st, dp, e, de, C, B,
                     H);
  return hipGetLastError();
}

hipError_t launch_up_back(Tensor du, Tensor d, Tensor dd, int C, int B, int H, hipStream_t st) {
  const int64_t n = (int64_t)B * H * H * (C / 8);
  hipLaunchKernelGGL(up_back_kernel, dim3(blocks256(n)), dim3(256), 0, st, du, d, dd, C, B, H);
  return hipGetLastError();
}

hipError_t launch_head(Tensor d, int C, const float* head, const float* u, double in_scale,
                       float* x0, int64_t npx, hipStream_t st) {
  hipLaunchKernelGGL(head_kernel, dim3(blocks256(npx)), dim3(256), 0, st, d, C, head, u,
                     (float)in_scale, x0, npx);
  return hipGetLastError();
}

// workgroups of the head's backward: at most 1024, each lane then covers
// every (1024 * 256)-th pixel
static unsigned head_blocks(int64_t npx) { return (unsigned)std::min<int64_t>(1024, blocks256(npx)); }

size_t head_part_doubles(int C, int64_t npx) { return (size_t)head_blocks(npx) * (C + 3); }

hipError_t launch_head_back(Tensor d, int C, const float* head, const float* u, double in_scale,
                            const float* x0, const float* target, int64_t npx, Tensor dz,
                            double* part, double* loss, float* dhead, hipStream_t st) {
  const unsigned nblk = head_blocks(npx);
  hipLaunchKernelGGL(head_back_kernel, dim3(nblk), dim3(256), (size_t)4 * (C + 3) * sizeof(double),
                     st, d, C, head, u, (float)in_scale, x0, target, npx, dz, part);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(head_reduce_kernel, dim3(C + 3), dim3(256), 0, st, (const double*)part,
                     (int)nblk, C, loss, dhead, 1.0 / (double)npx);
  return hipGetLastError();
}

hipError_t launch_adam(float* p, const float* g, float* m, float* v, int64_t n, float beta1,
                       float beta2, float lr_t, float eps_t, hipStream_t st) {
  hipLaunchKernelGGL(adam_kernel, dim3(blocks256(n)), dim3(256), 0, st, p, g, m, v, n, beta1,
                     beta2, lr_t, eps_t);
  return hipGetLastError();
}

hipError_t launch_cast_weights(const float* w, uint16_t* w16, uint16_t* wt16, int Cout, int Cin,
                               hipStream_t st) {
  const int64_t n = (int64_t)Cout * 9 * Cin;
  hipLaunchKernelGGL(cast_weights_kernel, dim3(blocks256(n)), dim3(256), 0, st, w, w16, wt16,
                     Cout, Cin);
  return hipGetLastError();
}

hipError_t launch_zero(float* x, int64_t n, hipStream_t st) {
  if (n <= 0) return hipSuccess;
  hipLaunchKernelGGL(zero_kernel, dim3(blocks256(n)), dim3(256), 0, st, x, n);
  return hipGetLastError();
}

}  // namespace cnn
}  // namespace slim
