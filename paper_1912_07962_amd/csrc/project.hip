// Matrix-free Joseph projectors for gfx950, for one slice or a batch of
// slices that share the geometry.
//
// Both kernels work on a tile of BT slices (BT = 1, 2 or 4, a template
// constant).  Global arrays stay slice-outer ([slice][N][N], [slice][list][R]);
// inside a workgroup the BT slices are interleaved in LDS, so the position of
// a ray in a row (forward) or the weights of a pixel (back) are computed once
// and applied to all BT slices with one 4/8/16-byte LDS read.
//
// Forward (ray-driven, LDS bands): the image is cut into bands of H rows
// (row-stepping angles) or H columns (column-stepping angles: H rows of the
// transposed image when the caller has one, else H columns of the image
// transposed on their way into LDS), H*(N+8)*BT floats <= 68 KB.  A
// workgroup owns a group of consecutive bands, a chunk of rays of one
// orientation and a slice tile; it streams its bands through LDS
// (zero-padded by four pixels on each side, so no bounds checks in the inner
// loop), prefetching the next band into registers, and every lane walks up
// to eight rays across them in pairs, interpolating linearly between the two
// pixels nearest the crossing point (Joseph).  The ray position is a 32.32
// fixed-point number; each wavefront walks the union of its rays' row ranges
// (wave-uniform loop).  Per-group partial sums are combined by a second
// kernel in a fixed order (deterministic, no atomics), which also applies
// h/d, subtracts the data and can fuse the CG tail.  Workgroups are numbered
// so that each XCD works on a contiguous range of (slice tile, band group)
// pairs, and the grid is sized to one round of resident workgroups (two per
// CU by default).
//
// Back (pixel-driven gather): a workgroup owns a 16 x 64 pixel tile (32 x 64
// without the update) of a slice tile and stages, for every angle of the list,
// the segment of ray values its tile touches (scaled by h/d) in LDS; each lane
// gathers two rays per angle for four pixels of a row, 16 columns apart, in
// each of its row blocks.  No atomics; the optional
// fused update writes x -= s, the transposed image, bf16 shadows and
// per-workgroup float64 partial norms.  Both projectors evaluate the same
// closed-form weights and agree to float32 rounding of the weights.
#include "slim_internal.h"
#include "pcg.h"

#include <algorithm>
#include <cstring>
#include <mutex>

namespace slim {

namespace {

// ---------------------------------------------------------------- helpers
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
__device__ __forceinline__ float comp(const float4& v, int k) {
  return k == 0 ? v.x : (k == 1 ? v.y : (k == 2 ? v.z : v.w));
}

// BT interleaved slices: one LDS element of BT floats
template <int BT> struct Lane;
template <> struct Lane<1> {
  typedef float T;
  static __device__ __forceinline__ float get(const float& v, int) { return v; }
};
template <> struct Lane<2> {
  typedef float2 T;
  static __device__ __forceinline__ float get(const float2& v, int b) { return b ? v.y : v.x; }
};
template <> struct Lane<4> {
  typedef float4 T;
  static __device__ __forceinline__ float get(const float4& v, int b) { return comp(v, b); }
};

// ---------------------------------------------------------------- forward
constexpr int kFT = 512;      // threads per forward workgroup
// Rays per lane, bounded by registers: every ray keeps a 32.32 position and
// step (4 VGPRs) and one fp64 accumulator per slice of the tile, and rays are
// walked in pairs, all within 128 VGPRs (four waves per SIMD: two 512-lane
// workgroups per CU).  More rays per workgroup means more angles per pass
// over the image, i.e. fewer passes.
constexpr int max_items(int BT) { return BT == 1 ? 8 : (BT == 2 ? 6 : 3); }
// the instantiated values: 1..6, then the cap
inline int item_count(int BT, int want) {
  const int it = want <= 6 ? want : 8;
  return it < max_items(BT) ? it : max_items(BT);
}
constexpr int kPad = 4;       // zero columns on each side of a band row (keeps rows 16B-aligned)
constexpr int kPF = 8;        // float4 prefetch registers per lane: H*N*BT/4 <= 8 * kFT

constexpr int kMaxOrd = 1024;   // largest grid whose chunk order is balanced

struct FwdPlan {
  int n;          // entries (= output rows)
  int n_row;      // entries 0..n_row-1 are row-stepping angles
  int per;        // rays per chunk (= items * threads per workgroup)
  int n_chunks;   // row-stepping chunks first
  int H, G;       // rows per band, bands per group
  int n_groups;
  int n_tiles;    // slice tiles of BT slices
  int items;      // rays per lane (template argument of the band kernel)
  int bt;         // slice tile (template argument of the band kernel)
  int il_lg;      // log2 of the number of angles whose rays interleave (ray_of)
  double inv_full;     // 1 / (2^il_lg R)
  double inv_tail[2];  // 1 / (angles left over after the interleaved groups), per orientation
  int n_ord;           // positions with a chunk in corder (0: chunk = position mod n_chunks)
  unsigned char corder[kMaxOrd];   // chunk of each position (a permutation within each tile-group)
  short id[kMaxList];
  short slot[kMaxList];
};

// Chunk c: rays [i0, i1) of one orientation group, counted from the group's
// first entry eg (ray i is entry eg + i / R, detector bin i % R).  Chunks may
// start and end inside an angle.
__device__ __forceinline__ void chunk_range(const FwdPlan& pl, int R, int c, int& eg, int& i0,
                                            int& i1, bool& colm) {
  const int nr = pl.n_row * R;
  const int nrc = (nr + pl.per - 1) / pl.per;
  colm = c >= nrc;
  eg = colm ? pl.n_row : 0;
  i0 = (colm ? c - nrc : c) * pl.per;
  i1 = min(colm ? (pl.n - pl.n_row) * R : nr, i0 + pl.per);
}

// Ray j of an orientation group of ng angles: the angles are taken in
// groups of il = 2^lg (il m ... il m + il - 1) whose rays interleave,
// j = il (m R + t) + (0 ... il - 1), so the 128 rays a wave walks together
// (a pair of 64-ray runs) are 128 / il detector bins of il angles adjacent in
// the list (within a block of the window: row ranges that differ little,
// and the bins' spread shrinks by il); the last ng mod il angles interleave
// likewise among themselves.
// floor(j / D) for 0 <= j < 2^24 and 1 <= D < 2^20 from inv = 1 / D rounded
// to double: j inv is within 2^-28 of j / D, whose fraction is 0 or at most
// 1 - 1/D < 1 - 2^-20, so adding 2^-21 before truncation gives the quotient.
__device__ __forceinline__ int div_by(int j, double inv) {
  return (int)fma((double)j, inv, 0x1p-21);
}

__device__ __forceinline__ void ray_of(int j, int ng, int R, int lg, double inv_full,
                                       double inv_tail, int& e, int& t) {
  const int il = 1 << lg, full = (ng >> lg) << lg;
  if (j < full * R) {
    const int m = div_by(j, inv_full), rem = j - m * il * R;
    e = il * m + (rem & (il - 1));
    t = rem >> lg;
  } else {
    const int j2 = j - full * R, k = ng - full;
    t = div_by(j2, inv_tail);
    e = full + j2 - t * k;
  }
}

// Ray of slot q of a lane within its chunk: slots 2p and 2p+1 of wave w hold
// rays 2p kFT + 128 w + [0, 64) and that + 64; an unpaired last slot (odd IT)
// holds (IT - 1) kFT + lane.  Every ray of the chunk is held exactly once.
template <int IT>
__device__ __forceinline__ int slot_item(int q, int tid) {
  if (q < IT - (IT & 1)) return (q >> 1) * 2 * kFT + (tid >> 6) * 128 + (q & 1) * 64 + (tid & 63);
  return q * kFT + tid;
}

// XCD-aware numbering of a launch's workgroups (the grid is a multiple of 8):
// consecutive positions (same slice tile and band group, different angle
// chunks) live on one XCD.
__device__ __forceinline__ int xcd_position() {
  const int per_xcd = gridDim.x >> 3;
  return (blockIdx.x & 7) * per_xcd + (blockIdx.x >> 3);
}

// The band kernel's work at position pos < n_groups n_chunks n_tiles of its
// plan (shared by the one-context launch and the grouped launch).
template <int IT, int BT, typename IMG>
__device__ __forceinline__ void fwd_band_body(int pos, const AngleGeom* __restrict__ geom, int N,
                                              int R, const FwdPlan& pl, int B,
                                              const IMG* __restrict__ img,
                                              const IMG* __restrict__ imgT, size_t img_stride,
                                              float* __restrict__ partial,
                                              const int* __restrict__ stop, int stop_stride) {
  typedef typename Lane<BT>::T LT;
  extern __shared__ float band[];
  const int W = N + 2 * kPad;
  const int chunk = pl.n_ord ? (int)pl.corder[pos] : pos % pl.n_chunks;
  const int tg = pos / pl.n_chunks;
  const int grp = tg % pl.n_groups;
  const int tile = tg / pl.n_groups;
  const int b0 = tile * BT;
  const int nb = min(BT, B - b0);
  if (stop) {
    bool all = true;
    for (int b = 0; b < nb; ++b) all = all && stop[(size_t)(b0 + b) * stop_stride + kCtlDone] != 0;
    if (all) return;
  }
  int eg, i0, i1;
  bool colm;
  chunk_range(pl, R, chunk, eg, i0, i1, colm);
  const int nitems = i1 - i0;
  const int ng = colm ? pl.n - pl.n_row : pl.n_row;   // angles of the orientation group
  // Column-stepping chunks walk the transposed image: from imgT when given
  // (bands of its rows), else from img as bands of columns, transposed on
  // their way into LDS.
  const bool cband = colm && imgT == nullptr;
  const IMG* src[BT];
#pragma unroll
  for (int b = 0; b < BT; ++b)
    src[b] = (colm && !cband ? imgT : img) + (size_t)(b0 + min(b, nb - 1)) * img_stride;
  const int kg = grp * pl.G * pl.H;

  // Ray position along the minor axis in 32.32 fixed point: P = pos * 2^32
  // at row k is P0 + k * S (pos: 0-based pixel index shifted by kPad).
  // Rounding P0 and S costs at most (k+1) * 2^-33 < 1.2e-7 pixel at k = 1023.
  // Each wavefront walks, per ray slot, the union of its 64 rays' row ranges
  // (a wave-uniform loop); a lane outside its own ray's range reads the zero
  // pads (its index is clamped into [0, W-2]) and adds nothing.  Slots are
  // walked in pairs, so a wave's two slots of a pair hold neighbouring runs
  // of 64 rays (similar row ranges); an unpaired last slot takes 64
  // consecutive rays per wave.
  int64_t P0[IT], S[IT];
  double acc[IT][BT];
  int wlo[IT], whi[IT];
  int oi[IT];   // the slot's output offset slot(e) R + t, -1 for no ray
  {
    // every slot first finds its ray (an empty slot takes the chunk's last
    // ray and is switched off below), so the table reads of all slots are
    // in flight together
    int e_[IT], t_[IT], id_[IT];
#pragma unroll
    for (int q = 0; q < IT; ++q) {
      const int item = min(slot_item<IT>(q, threadIdx.x), nitems - 1);
      ray_of(i0 + item, ng, R, pl.il_lg, pl.inv_full, pl.inv_tail[colm ? 1 : 0], e_[q], t_[q]);
      e_[q] += eg;
      id_[q] = pl.id[e_[q]];
    }
    const double lo_p = kPad - 1.5, hi_p = N + kPad + 0.5;
#pragma unroll
    for (int q = 0; q < IT; ++q) {
      const AngleGeom* g = geom + id_[q];
      const double inv = g->f_inv, c0 = g->f_c0, n1 = g->f_n1;
      const double qa = g->f_qa, qb = g->f_qb, qs = g->f_qs;
      const int64_t Sq = g->f_S;
      const bool live = slot_item<IT>(q, threadIdx.x) < nitems;
#pragma unroll
      for (int b = 0; b < BT; ++b) acc[q][b] = 0.0;
      const double tt = (double)t_[q];
      const double p0 = fma(tt, inv, c0);
      // rows with pos - kPad in [-1.5, N + 0.5] hold every contributing row
      double lo = 0.0, hi = N - 1;
      if (n1 != 0.0) {
        const double ma = fma(tt, qs, qa), mb = fma(tt, qs, qb);
        lo = fmax(lo, ceil(fmin(ma, mb)));
        hi = fmin(hi, floor(fmax(ma, mb)));
      } else if (p0 < lo_p || p0 > hi_p) {
        lo = 1.0;
        hi = 0.0;
      }
      int klo = N, khi = -1;
      if (live && lo <= hi) {
        klo = (int)lo;
        khi = (int)hi;
      }
      // index 0 (a pad column) and no step for an empty slot
      P0[q] = live ? __double2ll_rn(p0 * 4294967296.0) : 0;
      S[q] = live ? Sq : 0;
      oi[q] = live ? pl.slot[e_[q]] * R + t_[q] : -1;
      for (int o = 32; o > 0; o >>= 1) {
        klo = min(klo, __shfl_xor(klo, o, 64));
        khi = max(khi, __shfl_xor(khi, o, 64));
      }
      wlo[q] = __builtin_amdgcn_readfirstlane(klo);
      whi[q] = __builtin_amdgcn_readfirstlane(khi);
    }
  }

  // the zero pads are written once; band loads never touch them
  for (int e = threadIdx.x; e < pl.H * 2 * kPad * BT; e += kFT) {
    const int r = e / (2 * kPad * BT), c = (e / BT) % (2 * kPad), b = e % BT;
    band[(r * W + (c < kPad ? c : N + c)) * BT + b] = 0.f;
  }
  // Bands are software-pipelined: the next band's rows (BT slices, 16-byte
  // loads) are fetched into registers while the current band is used.  A
  // band of rows [k, k + h) is h N / 4 four-pixel chunks: chunk e is row
  // k + e / (N/4), columns 4 (e mod N/4) + [0, 4).  A band of columns (k and
  // h multiples of 4, see make_plan) is read in blocks of RB image rows x 4
  // columns: block e covers rows RB (e / (h/4)) + [0, RB), columns
  // k + 4 (e mod h/4) + [0, 4), so a wave reads whole row segments, and is
  // transposed in registers into runs of RB consecutive positions of each
  // column for the LDS writes.
  const bool vec = (N & 3) == 0 && (!cband || (pl.H & 3) == 0);
  const int n4 = N >> 2;
  constexpr int U = kPF / BT;  // 4-pixel chunks per lane per band
  constexpr int RB = U < 4 ? U : 4;
  constexpr int NBL = U / RB;  // column blocks per lane per band
  float4 pf[kPF];
  auto fetch_band = [&](int k, int h) {
    if (!cband) {
      const int lim = h * n4 - 1;
#pragma unroll
      for (int u = 0; u < U; ++u) {
        const int e = min((int)threadIdx.x + u * kFT, lim);
#pragma unroll
        for (int b = 0; b < BT; ++b) pf[u * BT + b] = load4(src[b], k * n4 + e);
      }
    } else {
      const int h4 = h >> 2, lim = (N / RB) * h4 - 1;
#pragma unroll
      for (int sb = 0; sb < NBL; ++sb) {
        const int e = min((int)threadIdx.x + sb * kFT, lim);
        const int i0 = RB * (e / h4), at = (k >> 2) + e % h4;
#pragma unroll
        for (int r = 0; r < RB; ++r) {
#pragma unroll
          for (int b = 0; b < BT; ++b) pf[(sb * RB + r) * BT + b] = load4(src[b], (i0 + r) * n4 + at);
        }
      }
    }
  };
  if (vec && kg < N) fetch_band(kg, min(pl.H, N - kg));
  for (int bb = 0; bb < pl.G; ++bb) {
    const int kb = kg + bb * pl.H;
    if (kb >= N) break;
    const int hb = min(pl.H, N - kb);
    __syncthreads();
    if (vec && !cband) {
      const int lim = hb * n4;
#pragma unroll
      for (int u = 0; u < U; ++u) {
        const int e = (int)threadIdx.x + u * kFT;
        const int r = e / n4, c4 = e - r * n4;
        if (e < lim) {
          float* dst = band + (size_t)(r * W + kPad + 4 * c4) * BT;
          if (BT == 1) {
            *reinterpret_cast<float4*>(dst) = pf[u];
          } else {
            // interleave: pixel k of the chunk holds the BT slices' values
#pragma unroll
            for (int k = 0; k < 4; ++k) {
#pragma unroll
              for (int b = 0; b < BT; ++b) dst[k * BT + b] = comp(pf[u * BT + b], k);
            }
          }
        }
      }
    } else if (vec) {
      const int h4 = hb >> 2, nbk = (N / RB) * h4;
#pragma unroll
      for (int sb = 0; sb < NBL; ++sb) {
        const int e = (int)threadIdx.x + sb * kFT;
        if (e < nbk) {
          const int i0 = RB * (e / h4), c4 = e % h4;
          // image rows i0 + r, columns kb + 4 c4 + k: band row 4 c4 + k,
          // positions i0 + r (RB BT consecutive floats, 16-byte aligned)
#pragma unroll
          for (int k = 0; k < 4; ++k) {
            float run[RB * BT];
#pragma unroll
            for (int r = 0; r < RB; ++r) {
#pragma unroll
              for (int b = 0; b < BT; ++b) run[r * BT + b] = comp(pf[(sb * RB + r) * BT + b], k);
            }
            float4* dst = reinterpret_cast<float4*>(band + (size_t)((4 * c4 + k) * W + kPad + i0) * BT);
#pragma unroll
            for (int q = 0; q < RB * BT / 4; ++q)
              dst[q] = make_float4(run[4 * q], run[4 * q + 1], run[4 * q + 2], run[4 * q + 3]);
          }
        }
      }
    } else if (!cband) {
      for (int e = threadIdx.x; e < hb * N * BT; e += kFT) {
        const int r = e / (N * BT), c = (e / BT) % N, b = e % BT;
        band[(r * W + kPad + c) * BT + b] = tof(src[b][(size_t)(kb + r) * N + c]);
      }
    } else {
      // element e: image row e / (hb BT), column kb + (e / BT) mod hb
      for (int e = threadIdx.x; e < hb * N * BT; e += kFT) {
        const int i = e / (hb * BT), r = (e / BT) % hb, b = e % BT;
        band[(r * W + kPad + i) * BT + b] = tof(src[b][(size_t)i * N + kb + r]);
      }
    }
    __syncthreads();
    const int kbn = kb + pl.H;
    if (vec && bb + 1 < pl.G && kbn < N) fetch_band(kbn, min(pl.H, N - kbn));
    const LT* bandv = reinterpret_cast<const LT*>(band);
    // Items walk the band in pairs over the union of their two row ranges,
    // so each row issues two independent LDS reads.  A lane outside its own
    // ray's range reads the zero pads (see above) and adds nothing.
#pragma unroll
    for (int q = 0; q < IT; q += 2) {
      const bool two = q + 1 < IT;   // known once unrolled
      const int qn = two ? q + 1 : q;
      const int k0 = max(min(wlo[q], wlo[qn]), kb), k1 = min(max(whi[q], whi[qn]), kb + hb - 1);
      if (k0 > k1) continue;  // wave-uniform
      int64_t Pa = P0[q] + (int64_t)k0 * S[q];
      int64_t Pb = P0[qn] + (int64_t)k0 * S[qn];
      const LT* row = bandv + (k0 - kb) * W;
      // sum over rows of a + phi (c - a), phi = lo(P) 2^-32, kept as the two
      // sums  sum a  and  sum lo(P) (c - a)  (the 2^-32 applied once per band)
      float aa[BT], da[BT], ab[BT], db[BT];
#pragma unroll
      for (int b = 0; b < BT; ++b) aa[b] = da[b] = ab[b] = db[b] = 0.f;
      // an index below 0 wraps above W - 2: both ends are zero pads
      auto fetch = [&](int64_t pa, int64_t pb, const LT* rw, LT& x0, LT& x1, LT& y0, LT& y1) {
        const uint32_t ia = min((uint32_t)(pa >> 32), (uint32_t)(W - 2));
        x0 = rw[ia];
        x1 = rw[ia + 1];
        y0 = x0;
        y1 = x1;
        if (two) {
          const uint32_t ib = min((uint32_t)(pb >> 32), (uint32_t)(W - 2));
          y0 = rw[ib];
          y1 = rw[ib + 1];
        }
      };
      auto add_row = [&](const LT& x0v, const LT& x1v, const LT& y0v, const LT& y1v, float la,
                         float lb) {
#pragma unroll
        for (int b = 0; b < BT; ++b) {
          const float x0 = Lane<BT>::get(x0v, b), x1 = Lane<BT>::get(x1v, b);
          aa[b] += x0;
          da[b] = fmaf(la, x1 - x0, da[b]);
          if (two) {
            const float y0 = Lane<BT>::get(y0v, b), y1 = Lane<BT>::get(y1v, b);
            ab[b] += y0;
            db[b] = fmaf(lb, y1 - y0, db[b]);
          }
        }
      };
      // pipelined by one row: the reads of row k + 1 are issued before the
      // sums of row k, so they are in flight while those run
      LT va0, va1, vb0, vb1;
      fetch(Pa, Pb, row, va0, va1, vb0, vb1);
      float la = (float)(uint32_t)Pa, lb = (float)(uint32_t)Pb;
      for (int k = k0; k < k1; ++k) {
        Pa += S[q];
        if (two) Pb += S[qn];
        // one position register per ray: keeps the compiler from carrying
        // the low word separately (extra 64-bit adds per row)
        asm volatile("" : "+v"(Pa), "+v"(Pb));
        row += W;
        LT na0, na1, nb0, nb1;
        fetch(Pa, Pb, row, na0, na1, nb0, nb1);
        const float nla = (float)(uint32_t)Pa, nlb = (float)(uint32_t)Pb;
        add_row(va0, va1, vb0, vb1, la, lb);
        va0 = na0;
        va1 = na1;
        vb0 = nb0;
        vb1 = nb1;
        la = nla;
        lb = nlb;
      }
      add_row(va0, va1, vb0, vb1, la, lb);
#pragma unroll
      for (int b = 0; b < BT; ++b) {
        acc[q][b] += (double)fmaf(da[b], 2.3283064365386963e-10f, aa[b]);
        if (two) acc[qn][b] += (double)fmaf(db[b], 2.3283064365386963e-10f, ab[b]);
      }
    }
  }
#pragma unroll
  for (int q = 0; q < IT; ++q) {
    if (oi[q] >= 0) {
#pragma unroll
      for (int b = 0; b < BT; ++b)
        if (b < nb)
          partial[((size_t)(b0 + b) * pl.n_groups + grp) * pl.n * R + oi[q]] = (float)acc[q][b];
    }
  }
}

template <int IT, int BT, typename IMG>
__global__ __launch_bounds__(kFT, 2) void fwd_band_kernel(const AngleGeom* __restrict__ geom, int N,
                                                          int R, FwdPlan pl, int B,
                                                          const IMG* __restrict__ img,
                                                          const IMG* __restrict__ imgT,
                                                          size_t img_stride,
                                                          float* __restrict__ partial,
                                                          const int* __restrict__ stop,
                                                          int stop_stride) {
  const int pos = xcd_position();
  if (pos >= pl.n_groups * pl.n_chunks * pl.n_tiles) return;
  fwd_band_body<IT, BT, IMG>(pos, geom, N, R, pl, B, img, imgT, img_stride, partial, stop,
                             stop_stride);
}

// out[s][t] = (h/d) sum_groups partial - sub for slice sl (ray block bx of
// 256); optional CG tail q = out + lam*pd with per-workgroup partial dots
// <pd, q> (and <pd, pd> into dots2 when it is non-NULL).
template <typename SUB>
__device__ __forceinline__ void fwd_reduce_body(
    int bx, int sl, const AngleGeom* __restrict__ geom, int R, const AngleList& ids, int n_groups,
    const float* __restrict__ partial, const SUB* __restrict__ sub, size_t sub_stride,
    float* __restrict__ out32, double* __restrict__ out64, size_t out_stride,
    const double* __restrict__ pd, size_t pd_stride, double lam, double* __restrict__ dots,
    double* __restrict__ dots2, size_t dots_stride, const int* __restrict__ stop,
    int stop_stride) {
  // the stop flag is read with everything else; a stopped slice's
  // workgroups leave before writing
  const bool stopped = stop && stop[(size_t)sl * stop_stride + kCtlDone];
  __shared__ double sh[8];
  const int o = bx * 256 + threadIdx.x;
  const int n = ids.n * R;
  double d = 0.0, d2 = 0.0;
  if (o < n) {
    const int s = o / R, t = o % R;
    const int ang = ids.id[s];
    const size_t gs = (size_t)ids.n * R;
    const float* pp = partial + (size_t)sl * n_groups * gs + (size_t)s * R + t;
    // band groups summed in order, loaded 16 at a time without branches
    // (past the last group: the last one is read again and +0 added)
    constexpr int kLd = 16;
    double v = 0.0;
    for (int g = 0; g < n_groups; g += kLd) {
      float a[kLd];
#pragma unroll
      for (int u = 0; u < kLd; ++u) a[u] = pp[(size_t)min(g + u, n_groups - 1) * gs];
#pragma unroll
      for (int u = 0; u < kLd; ++u) v += g + u < n_groups ? (double)a[u] : 0.0;
    }
    if (stopped) return;   // the same for the whole workgroup
    v *= (double)geom[ang].hd;
    if (sub) v -= (double)tof(sub[(size_t)sl * sub_stride + (size_t)ang * R + t]);
    if (pd) {
      const double pv = pd[(size_t)sl * pd_stride + o];
      v = fma(lam, pv, v);
      // rounded products (never fused into the sums below), so every
      // launch that runs this body forms the same dot products
      d = __dmul_rn(pv, v);
      d2 = __dmul_rn(pv, pv);
    }
    if (out32) out32[(size_t)sl * out_stride + o] = (float)v;
    if (out64) out64[(size_t)sl * out_stride + o] = v;
  } else if (stopped) {
    return;
  }
  if (dots) {
    for (int w = 32; w > 0; w >>= 1) {
      d += __shfl_down(d, w, 64);
      d2 += __shfl_down(d2, w, 64);
    }
    if ((threadIdx.x & 63) == 0) {
      sh[threadIdx.x >> 6] = d;
      sh[4 + (threadIdx.x >> 6)] = d2;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
      dots[(size_t)sl * dots_stride + bx] = sh[0] + sh[1] + sh[2] + sh[3];
      if (dots2) dots2[(size_t)sl * dots_stride + bx] = sh[4] + sh[5] + sh[6] + sh[7];
    }
  }
}

template <typename SUB>
__global__ __launch_bounds__(256) void fwd_reduce_kernel(
    const AngleGeom* __restrict__ geom, int R, AngleList ids, int n_groups,
    const float* __restrict__ partial, const SUB* __restrict__ sub, size_t sub_stride,
    float* __restrict__ out32, double* __restrict__ out64, size_t out_stride,
    const double* __restrict__ pd, size_t pd_stride, double lam, double* __restrict__ dots,
    double* __restrict__ dots2, size_t dots_stride, const int* __restrict__ stop,
    int stop_stride) {
  fwd_reduce_body<SUB>(blockIdx.x, blockIdx.y, geom, R, ids, n_groups, partial, sub, sub_stride,
                       out32, out64, out_stride, pd, pd_stride, lam, dots, dots2, dots_stride,
                       stop, stop_stride);
}

// ------------------------------------------------------------------- back
constexpr int kBH = 16, kBW = 64;   // tile rows, columns (per row block of 16)
constexpr int kBPX = 4;             // pixels per lane and row block
// rays of one angle's segment: the detector span of a 32 x 64 tile (two row
// blocks) is at most sqrt(31^2 + 63^2) < 71 ray spacings between its corner
// pixels, plus the floor, the next ray and the segment's first-ray margin
constexpr int kSeg = 80;
constexpr int kSegFloats = 64 * kSeg;   // LDS floats of staged segments
constexpr int kPre = kSegFloats / 512;  // staged values per lane per pass (two buffers)

// Per-angle constants of one staged pass, positions in 32.32 fixed point.
// T0 is the canonical detector coordinate of the tile's first pixel moved by
// an integer onto the angle's LDS segment (segment index = ray - tmin +
// a * kSeg), split into (segment index of ray floor(t), fraction); Ts and Tc
// step one row and one column; step = kQ Tc is the distance between a
// lane's pixels; invd32 = 2^-32 / d.
struct BackAngle {
  uint64_t T0;
  int64_t Ts, Tc;
  int64_t step;
  int64_t rstep;   // 16 Ts: the lane's next row block
  float invd32, c1;
};

// min(max(x, 0), 1): the weights are at most 1 by construction, so this is
// max(0, x); written as a median it folds into the producing instruction's
// output clamp.
__device__ __forceinline__ float unit_clamp(float x) { return __builtin_amdgcn_fmed3f(x, 0.f, 1.f); }

__device__ __forceinline__ double wave_sum(double v) {
  for (int o = 32; o > 0; o >>= 1) v += __shfl_down(v, o, 64);
  return v;
}

// The back-projector's work for pixel tile (bx, by) of a gx x gy grid of
// tiles and slice tile bz (shared by the one-context launch and the grouped
// launch).  A tile is 16 RB rows by 64 columns: a lane's pixels are rows
// ty + 16 r (r < RB) of columns tx + 16 q (q < 4).
template <typename VT, int BT, int RB>
__device__ __forceinline__ void back_body(
    int bx, int by, int bz, int gx, int gy, const AngleGeom* __restrict__ geom, int N, int R,
    const AngleList& ids, int B, const VT* __restrict__ v, size_t v_stride,
    float* __restrict__ out, float* __restrict__ x, float* __restrict__ xT,
    const float* __restrict__ x_true, size_t img_stride, double* __restrict__ partials, int mode,
    const int* __restrict__ stop, int stop_stride, uint16_t* __restrict__ xs,
    uint16_t* __restrict__ xsT, float shrink) {
  typedef typename Lane<BT>::T LT;
  // A lane's pixels are columns tx + 16 q: for each q the 16 lanes of a row
  // take consecutive columns, so a wave's LDS reads hit nearby rays (fewer
  // bank conflicts than four consecutive pixels per lane, whose lanes' reads
  // spread over four times the rays; measured 20-25% faster).
  constexpr int kQ = 16;     // columns between a lane's pixels
  constexpr int kL = 1;      // columns between lanes
  // One slice: the LDS segments form two pass buffers, the next pass loaded
  // into registers and stored while the current one is used.  Slice tiles:
  // one buffer of more angles, staged between barriers (the lanes' LDS reads,
  // not load latency, bound those).
  constexpr bool kDB = BT == 1;
  constexpr int kBuf = kDB ? kSegFloats / 2 : kSegFloats;  // floats of one pass buffer
  constexpr int kPass = kBuf / (kSeg * BT);               // angles staged per pass
  constexpr int kConst = kDB ? kMaxList : kPass;           // angles with constants held
  const int b0 = bz * BT;
  const int nb = min(BT, B - b0);
  if (stop) {
    bool all = true;
    for (int b = 0; b < nb; ++b) all = all && stop[(size_t)(b0 + b) * stop_stride + kCtlDone] != 0;
    if (all) return;
  }
  __shared__ float seg[kSegFloats];
  __shared__ int tmin[kConst];
  __shared__ float hdA[kConst];
  __shared__ BackAngle ang[kConst];
  __shared__ double wred[4][3 * BT];
  // the transposed-copy tile reuses the segment buffers once every pass is done
  constexpr int kTH = kBH * RB;           // tile rows
  static_assert(kSegFloats >= kTH * (kBW + 1), "tile does not fit the segment buffers");
  float(*tile)[kBW + 1] = reinterpret_cast<float(*)[kBW + 1]>(seg);
  const int tx = threadIdx.x & 15;       // 16 lanes x 4 pixels = 64 columns
  const int ty = threadIdx.x >> 4;       // 16 rows per row block
  const int i0 = by * kTH, j0 = bx * kBW;
  const int i = i0 + ty;                 // the lane's row in row block r: i + 16 r
  const int jb = j0 + kL * tx;           // pixel q of the lane: column jb + kQ q
  const double half = 0.5 * (N - 1);
  // detector coordinates are shifted by kTOff (>= every |jj c + ii s|), so
  // they are positive and float->int truncation is floor
  const int kTOff = 2 * N + 8;
  const double off = 0.5 * (R - 1) + kTOff;
  // nominal tile corners (pixel centres) bound every pixel the lanes evaluate
  const double ci0 = (double)i0 - half, ci1 = (double)(i0 + kTH - 1) - half;
  const double cj0 = (double)j0 - half, cj1 = (double)(j0 + kBW - 1) - half;
  // constants of list angle a in slot c: the first ray of its segment (tmin)
  // and the position constants (base relative to its place in the pass)
  auto set_const = [&](int a, int c) {
    const AngleGeom g = geom[ids.id[a]];
    const double t00 = det_coord(g, ci0, cj0, off), t01 = det_coord(g, ci0, cj1, off);
    const double t10 = det_coord(g, ci1, cj0, off), t11 = det_coord(g, ci1, cj1, off);
    const int tm = (int)floor(fmin(fmin(t00, t01), fmin(t10, t11))) - 1;
    tmin[c] = tm;
    hdA[c] = g.hd;
    BackAngle A;
    {
      // integer and fraction of the corner's coordinate taken before the
      // (integer) move onto the segment, so the fraction does not depend on
      // the pass layout (slice tile) and no rounding of the moved sum enters
      const double t = det_coord(g, ci0, cj0, off);
      const double fl = floor(t);
      const int t0 = (int)fl + (a % kPass) * kSeg - tm;   // >= 1
      A.T0 = ((uint64_t)(uint32_t)t0 << 32) | (uint32_t)((t - fl) * 4294967296.0);
    }
    A.Ts = __double2ll_rn(g.s * 4294967296.0);
    A.Tc = __double2ll_rn(g.c * 4294967296.0);
    A.step = kQ * A.Tc;
    A.rstep = kBH * A.Ts;
    A.invd32 = g.invd * 2.3283064365386963e-10f;
    A.c1 = 1.f - g.invd;
    ang[c] = A;
  };
  float s[RB * kBPX][BT];   // pixel (r, q) at index r kBPX + q
#pragma unroll
  for (int q = 0; q < RB * kBPX; ++q)
#pragma unroll
    for (int b = 0; b < BT; ++b) s[q][b] = 0.f;
  // na angles of a pass from LDS segments segp, constants from slot c0
  // (rows past the image are evaluated too when RB > 1: their positions lie
  // within the tile's nominal corners, so inside the segments)
  auto accumulate = [&](const float* segp, int c0, int na) {
    if (RB == 1 && i >= N) return;
    const LT* segv = reinterpret_cast<const LT*>(segp);
    for (int a = 0; a < na; ++a) {
      const BackAngle A = ang[c0 + a];
      // the lane's first pixel (row ty, column tx of the tile); with the
      // steps to its other pixels every position is within 56 2^-32
      // (< 2e-8 pixel) of the canonical coordinate
      uint64_t Tr = A.T0 + (uint64_t)((int64_t)ty * A.Ts) + (uint64_t)((int64_t)tx * A.Tc);
#pragma unroll
      for (int r = 0; r < RB; ++r) {
        if (r) Tr += (uint64_t)A.rstep;           // 16 rows on: t + 16 s
        uint64_t T = Tr;
#pragma unroll
        for (int q = 0; q < kBPX; ++q) {
          if (q) T += (uint64_t)A.step;           // kQ columns on: t + kQ c
          const uint32_t k = (uint32_t)(T >> 32);
          const float f = (float)(uint32_t)T;     // 2^32 x distance to ray k
          const float w0 = unit_clamp(fmaf(-f, A.invd32, 1.f));   // 1 - f/d
          const float w1 = unit_clamp(fmaf(f, A.invd32, A.c1));   // 1 - (1-f)/d
          const LT v0 = segv[k], v1 = segv[k + 1];
#pragma unroll
          for (int b = 0; b < BT; ++b)
            s[r * kBPX + q][b] =
                fmaf(w0, Lane<BT>::get(v0, b), fmaf(w1, Lane<BT>::get(v1, b), s[r * kBPX + q][b]));
        }
      }
    }
  };
  // Staged value e of a pass starting at list angle a0: angle a0 + e / (kSeg
  // BT), segment ray (e / BT) % kSeg, slice e % BT; tmin and h/d from slot
  // cs(a) of the angle; rays outside [0, R) stage 0.
  const int npass = (ids.n + kPass - 1) / kPass;
  if constexpr (kDB) {
    for (int a = threadIdx.x; a < ids.n; a += 256) set_const(a, a);
    __syncthreads();
    // register-held loads of a pass (ray index clamped into the row; the
    // value is scaled, or zeroed, when stored)
    VT pf[kPre];
    auto fetch = [&](int p) {
      const int a0 = p * kPass, n_e = min(kPass, ids.n - a0) * kSeg * BT;
#pragma unroll
      for (int u = 0; u < kPre; ++u) {
        const int e = (int)threadIdx.x + u * 256;
        if (e < n_e) {
          const int a = a0 + e / (kSeg * BT), b = e % BT;
          const int t = min(max(tmin[a] + (e / BT) % kSeg - kTOff, 0), R - 1);
          pf[u] = v[(size_t)(b0 + min(b, nb - 1)) * v_stride + (size_t)a * R + t];
        }
      }
    };
    auto store = [&](int p) {
      float* dst = seg + (p & 1) * kBuf;
      const int a0 = p * kPass, n_e = min(kPass, ids.n - a0) * kSeg * BT;
#pragma unroll
      for (int u = 0; u < kPre; ++u) {
        const int e = (int)threadIdx.x + u * 256;
        if (e < n_e) {
          const int a = a0 + e / (kSeg * BT);
          const int t = tmin[a] + (e / BT) % kSeg - kTOff;
          dst[e] = (t >= 0 && t < R) ? hdA[a] * (float)pf[u] : 0.f;
        }
      }
    };
    fetch(0);
    store(0);
    if (npass > 1) fetch(1);
    __syncthreads();
    for (int p = 0; p < npass; ++p) {
      accumulate(seg + (p & 1) * kBuf, p * kPass, min(kPass, ids.n - p * kPass));
      if (p + 1 < npass) {
        store(p + 1);   // the other buffer: its last readers passed the previous barrier
        if (p + 2 < npass) fetch(p + 2);
      }
      __syncthreads();
    }
  } else {
    for (int p = 0; p < npass; ++p) {
      const int a0 = p * kPass, na = min(kPass, ids.n - a0);
      __syncthreads();
      if ((int)threadIdx.x < na) set_const(a0 + threadIdx.x, threadIdx.x);
      __syncthreads();
      // one independent global load per staged value (unrolled so several
      // are in flight per lane)
#pragma unroll 6
      for (int e = threadIdx.x; e < na * kSeg * BT; e += 256) {
        const int a = e / (kSeg * BT), b = e % BT;
        const int t = tmin[a] + (e / BT) % kSeg - kTOff;
        const VT* vb = v + (size_t)(b0 + min(b, nb - 1)) * v_stride;
        seg[e] = (t >= 0 && t < R) ? hdA[a] * (float)vb[(size_t)(a0 + a) * R + t] : 0.f;
      }
      __syncthreads();
      accumulate(seg, 0, na);
    }
    __syncthreads();   // the segments are reused as the transposed-copy tile
  }
  if (mode == 0) {
#pragma unroll
    for (int b = 0; b < BT; ++b) {
      if (b >= nb) break;
      float* ob = out + (size_t)(b0 + b) * img_stride;
#pragma unroll
      for (int r = 0; r < RB; ++r) {
        const int ir = i + kBH * r;
        if (ir < N) {
#pragma unroll
          for (int q = 0; q < kBPX; ++q)
            if (jb + kQ * q < N) ob[(size_t)ir * N + jb + kQ * q] = s[r * kBPX + q][b];
        }
      }
      if (xT) {  // transposed copy of out through LDS
        __syncthreads();
#pragma unroll
        for (int r = 0; r < RB; ++r)
#pragma unroll
          for (int q = 0; q < kBPX; ++q) tile[ty + kBH * r][kL * tx + kQ * q] = s[r * kBPX + q][b];
        __syncthreads();
        float* tb = xT + (size_t)(b0 + b) * img_stride;
        for (int e = threadIdx.x; e < kTH * kBW; e += 256) {
          const int jl = e / kTH, il = e % kTH;
          if (j0 + jl < N && i0 + il < N) tb[(size_t)(j0 + jl) * N + i0 + il] = tile[il][jl];
        }
      }
    }
    return;
  }
  double nrm[BT][3];
#pragma unroll
  for (int b = 0; b < BT; ++b) {
    nrm[b][0] = nrm[b][1] = nrm[b][2] = 0.0;
    float xn[RB * kBPX];
#pragma unroll
    for (int q = 0; q < RB * kBPX; ++q) xn[q] = 0.f;
    if (b < nb) {
      const size_t so = (size_t)(b0 + b) * img_stride;
#pragma unroll
      for (int r = 0; r < RB; ++r) {
        const int ir = i + kBH * r;
        if (ir >= N) continue;
#pragma unroll
        for (int q = 0; q < kBPX; ++q) {
          if (jb + kQ * q < N) {
            const int pq = r * kBPX + q;
            const size_t p = so + (size_t)ir * N + jb + kQ * q;
            const float xo = x[p];
            const float sq = fmaf(shrink, xo, s[pq][b]);
            xn[pq] = xo - sq;
            x[p] = xn[pq];
            if (xs) xs[p] = f2bf(xn[pq]);
            nrm[b][0] += (double)sq * (double)sq;
            nrm[b][1] += (double)xn[pq] * (double)xn[pq];
            if (x_true) {
              const double e = (double)xn[pq] - (double)x_true[p];
              nrm[b][2] += e * e;
            }
          }
        }
      }
      if (xT || xsT) {
        __syncthreads();
#pragma unroll
        for (int r = 0; r < RB; ++r)
#pragma unroll
          for (int q = 0; q < kBPX; ++q) tile[ty + kBH * r][kL * tx + kQ * q] = xn[r * kBPX + q];
        __syncthreads();
        for (int e = threadIdx.x; e < kTH * kBW; e += 256) {
          const int jl = e / kTH, il = e % kTH;
          if (j0 + jl < N && i0 + il < N) {
            const size_t o = so + (size_t)(j0 + jl) * N + i0 + il;
            if (xT) xT[o] = tile[il][jl];
            if (xsT) xsT[o] = f2bf(tile[il][jl]);
          }
        }
      }
    }
  }
  const int w = threadIdx.x >> 6;
#pragma unroll
  for (int b = 0; b < BT; ++b)
#pragma unroll
    for (int k = 0; k < 3; ++k) {
      const double r = wave_sum(nrm[b][k]);
      if ((threadIdx.x & 63) == 0) wred[w][3 * b + k] = r;
    }
  __syncthreads();
  const int nwg = gx * gy;
  const int wg = by * gx + bx;
  if ((int)threadIdx.x < 3 * nb) {
    const int b = threadIdx.x / 3, k = threadIdx.x % 3;
    const double r = wred[0][threadIdx.x] + wred[1][threadIdx.x] + wred[2][threadIdx.x] +
                     wred[3][threadIdx.x];
    partials[((size_t)(b0 + b) * nwg + wg) * 3 + k] = r;
  }
}

template <typename VT, int BT, int RB>
__global__ __launch_bounds__(256) void back_kernel(
    const AngleGeom* __restrict__ geom, int N, int R, AngleList ids, int B,
    const VT* __restrict__ v, size_t v_stride, float* __restrict__ out, float* __restrict__ x,
    float* __restrict__ xT, const float* __restrict__ x_true, size_t img_stride,
    double* __restrict__ partials, int mode, const int* __restrict__ stop, int stop_stride,
    uint16_t* __restrict__ xs, uint16_t* __restrict__ xsT, float shrink) {
  back_body<VT, BT, RB>(blockIdx.x, blockIdx.y, blockIdx.z, gridDim.x, gridDim.y, geom, N, R, ids, B,
                    v, v_stride, out, x, xT, x_true, img_stride, partials, mode, stop, stop_stride,
                    xs, xsT, shrink);
}

// ------------------------------------------------------- grouped launches
// The CG products of several contexts (images of different sizes, the same
// angle list) in one launch per kernel: workgroup w finds its context g in a
// table of descriptors in device memory (start: the first workgroup or
// position of the context) and runs the one-context body at w - start.
// The band kernel's positions keep the XCD layout of a one-context launch:
// every XCD runs per = ceil(total / 8) consecutive positions of each
// context, its slots start .. start + per - 1 (of the launch's workgroups
// that the XCD runs) holding positions x per + (slot - start) on XCD x.
struct FwdGroupDesc {
  FwdPlan pl;
  const AngleGeom* geom;
  const float* img;
  const float* imgT;
  float* partial;
  const int* stop;
  size_t img_stride;
  int N, R, B, stop_stride, start, per, total, bt, items;
};

struct RedGroupDesc {
  AngleList ids;
  const AngleGeom* geom;
  const float* partial;
  double* out64;
  const double* pd;
  double* dots;
  double* dots2;
  const int* stop;
  size_t out_stride, pd_stride, dots_stride;
  double lam;
  int R, n_groups, gx, start, stop_stride;
};

struct BackGroupDesc {
  AngleList ids;
  const AngleGeom* geom;
  const double* v;
  float* out;
  float* xT;
  const int* stop;
  size_t v_stride, img_stride;
  int N, R, B, gx, gy, start, stop_stride;
};

template <typename D>
__device__ __forceinline__ int group_of(const D* __restrict__ d, int n, int w) {
  int g = 0;
  while (g + 1 < n && w >= d[g + 1].start) ++g;
  return g;
}

// every (slice tile, rays per lane) pair that launch_band instantiates
__global__ __launch_bounds__(kFT, 2) void fwd_band_grouped(const FwdGroupDesc* __restrict__ d,
                                                           int n) {
  const int xcd = blockIdx.x & 7, slot = blockIdx.x >> 3;
  const FwdGroupDesc& a = d[group_of(d, n, slot)];
  const int lp = xcd * a.per + (slot - a.start);
  if (lp >= a.total) return;
#define SLIM_GRP_CASE(BT_, IT_)                                                                 \
  case BT_ * 16 + IT_:                                                                          \
    fwd_band_body<IT_, BT_, float>(lp, a.geom, a.N, a.R, a.pl, a.B, a.img, a.imgT, a.img_stride, \
                                   a.partial, a.stop, a.stop_stride);                           \
    break;
  switch (a.bt * 16 + a.items) {
    SLIM_GRP_CASE(1, 1) SLIM_GRP_CASE(1, 2) SLIM_GRP_CASE(1, 3) SLIM_GRP_CASE(1, 4)
    SLIM_GRP_CASE(1, 5) SLIM_GRP_CASE(1, 6) SLIM_GRP_CASE(1, 8)
    SLIM_GRP_CASE(2, 1) SLIM_GRP_CASE(2, 2) SLIM_GRP_CASE(2, 3) SLIM_GRP_CASE(2, 4)
    SLIM_GRP_CASE(2, 5) SLIM_GRP_CASE(2, 6)
    SLIM_GRP_CASE(4, 1) SLIM_GRP_CASE(4, 2) SLIM_GRP_CASE(4, 3)
    default: break;
  }
#undef SLIM_GRP_CASE
}

__global__ __launch_bounds__(256) void fwd_reduce_grouped(const RedGroupDesc* __restrict__ d,
                                                          int n) {
  const int w = blockIdx.x;
  const RedGroupDesc& a = d[group_of(d, n, w)];
  const int lw = w - a.start;
  fwd_reduce_body<float>(lw % a.gx, lw / a.gx, a.geom, a.R, a.ids, a.n_groups, a.partial,
                         (const float*)nullptr, 0, nullptr, a.out64, a.out_stride, a.pd,
                         a.pd_stride, a.lam, a.dots, a.dots2, a.dots_stride, a.stop,
                         a.stop_stride);
}

template <int BT>
__global__ __launch_bounds__(256) void back_grouped(const BackGroupDesc* __restrict__ d, int n) {
  const int w = blockIdx.x;
  const BackGroupDesc& a = d[group_of(d, n, w)];
  const int lw = w - a.start;
  const int per = a.gx * a.gy;
  const int bz = lw / per, rem = lw - bz * per;
  back_body<double, BT, 2>(rem % a.gx, rem / a.gx, bz, a.gx, a.gy, a.geom, a.N, a.R, a.ids, a.B, a.v,
                        a.v_stride, a.out, nullptr, a.xT, nullptr, a.img_stride, nullptr, 0, a.stop,
                        a.stop_stride, nullptr, nullptr, 0.f);
}

// out[3*slice + k] = sum over n partial 3-vectors of the slice (fixed order)
__global__ __launch_bounds__(256) void reduce3_kernel(const double* __restrict__ partials, int n,
                                                      double* __restrict__ out) {
  __shared__ double red[3][256];
  const double* p = partials + (size_t)blockIdx.x * n * 3;
  double a0 = 0.0, a1 = 0.0, a2 = 0.0;
  for (int k = threadIdx.x; k < n; k += 256) {
    a0 += p[3 * (size_t)k + 0];
    a1 += p[3 * (size_t)k + 1];
    a2 += p[3 * (size_t)k + 2];
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
  if (threadIdx.x < 3) out[3 * (size_t)blockIdx.x + threadIdx.x] = red[threadIdx.x][0];
}

constexpr int kTile = 16;

// dst = src^T (float32, optional); bf16 copies of src and of src^T (optional);
// blockIdx.z = slice
__global__ __launch_bounds__(256) void transpose_kernel(const float* __restrict__ src,
                                                        float* __restrict__ dst, int N,
                                                        size_t stride,
                                                        uint16_t* __restrict__ bs,
                                                        uint16_t* __restrict__ bsT) {
  __shared__ float t[kTile][kTile + 1];
  const size_t so = (size_t)blockIdx.z * stride;
  const int tx = threadIdx.x & (kTile - 1), ty = threadIdx.x / kTile;
  const int i = blockIdx.y * kTile + ty, j = blockIdx.x * kTile + tx;
  if (i < N && j < N) {
    const float v = src[so + (size_t)i * N + j];
    t[ty][tx] = v;
    if (bs) bs[so + (size_t)i * N + j] = f2bf(v);
  }
  __syncthreads();
  const int jt = blockIdx.x * kTile + ty, it = blockIdx.y * kTile + tx;
  if (jt < N && it < N) {
    if (dst) dst[so + (size_t)jt * N + it] = t[tx][ty];
    if (bsT) bsT[so + (size_t)jt * N + it] = f2bf(t[tx][ty]);
  }
}

// out[s][i][t] = b[s][ids[i]][t]: rows of the sinogram for a list of angles
template <typename T>
__global__ __launch_bounds__(256) void gather_rows_kernel(const T* __restrict__ b, int n_angles,
                                                          int R, AngleList ids,
                                                          float* __restrict__ out) {
  const int i = blockIdx.y, s = blockIdx.z;
  const int t = blockIdx.x * 256 + threadIdx.x;
  if (t >= R) return;
  out[((size_t)s * ids.n + i) * R + t] = tof(b[((size_t)s * n_angles + ids.id[i]) * R + t]);
}

}  // namespace

// ---------------------------------------------------------------- launchers
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

int slice_tile(int B) { return B >= 4 ? 4 : (B >= 2 ? 2 : 1); }

// The forward projector's slice tile: as wide as the batch allows while a
// band still holds at least kMinRows image rows (the band is 64-68 KB of LDS,
// so wide tiles of large images would leave a few rows per barrier).
constexpr int kMinRows = 8;
static int fwd_slice_tile(int B, int N) {
  int bt = slice_tile(B);
  while (bt > 1 && 16384 / ((N + 2 * kPad) * bt) < kMinRows) bt >>= 1;
  return bt;
}

// Launch plan: rays grouped by orientation (row-stepping angles first) and
// cut into chunks of items * kFT rays, slices into tiles of BT, image bands
// into groups, with chunks * tiles * groups <= 2 * (number of
// CUs) where possible, so that a launch is one round of resident workgroups
// (two per CU, bounded by LDS).
void fwd_angle_consts(AngleGeom& g, int N, int R) {
  const bool colm = g.colmajor != 0;
  const double cm = colm ? g.c : g.s;   // coefficient of the major coordinate
  const double cn = colm ? g.s : g.c;   // of the minor one, |cn| = d
  const double half = 0.5 * (N - 1), off = 0.5 * (R - 1);
  const double inv = 1.0 / cn;
  const double n1 = -cm * inv;
  g.f_inv = inv;
  g.f_n1 = n1;
  g.f_c0 = half + kPad - half * n1 - off * inv;
  g.f_S = llrint(n1 * 4294967296.0);
  const double lo_p = kPad - 1.5, hi_p = N + kPad + 0.5;
  if (n1 != 0.0) {
    g.f_qa = (lo_p - g.f_c0) / n1;
    g.f_qb = (hi_p - g.f_c0) / n1;
    g.f_qs = -inv / n1;
  } else {
    g.f_qa = g.f_qb = g.f_qs = 0.0;
  }
}

static FwdPlan make_plan(const AngleGeom* h_geom, int N, int R, const AngleList& ids, int B,
                         const ProjTune& tune) {
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
  int BT = tune.fwd_bt > 0 ? std::min(tune.fwd_bt, slice_tile(B)) : fwd_slice_tile(B, N);
  // one band row of BT slices must fit the lanes' prefetch registers
  while (BT > 1 && (size_t)N * BT > (size_t)4 * kPF * kFT) BT >>= 1;
  pl.bt = BT;
  const int cap = tune.fwd_items > 0 ? std::min(tune.fwd_items, max_items(BT)) : max_items(BT);
  const int most = std::max(pl.n_row, ids.n - pl.n_row) * R;   // rays of the larger group
  pl.items = item_count(BT, std::max(1, std::min(cap, (most + kFT - 1) / kFT)));
  pl.per = pl.items * kFT;
  pl.n_chunks = (pl.n_row * R + pl.per - 1) / pl.per + ((ids.n - pl.n_row) * R + pl.per - 1) / pl.per;
  pl.n_tiles = (B + BT - 1) / BT;
  // interleaving more angles shrinks each wave's union of row ranges but
  // spreads its LDS reads over more clusters: four angles paid off for
  // detectors of 725 bins (512^2 volume window), two for 1449 (1024^2)
  pl.il_lg = R >= 1024 ? 1 : 2;
  pl.inv_full = 1.0 / (double)((1 << pl.il_lg) * R);
  for (int o = 0; o < 2; ++o) {
    const int ng = o ? ids.n - pl.n_row : pl.n_row;
    const int k = ng - ((ng >> pl.il_lg) << pl.il_lg);
    pl.inv_tail[o] = 1.0 / (double)(k > 0 ? k : 1);
  }
  pl.H = std::max(1, std::min(N, 16384 / ((N + 2 * kPad) * BT)));
  // bands of columns load four columns per 16-byte read: H a multiple of 4
  // (rounded up while the band stays within 68 KB and the lanes' prefetch
  // registers, else down), so every band starts at a multiple of 4 (the
  // last one may be shorter)
  if ((N & 3) == 0 && (pl.H & 3) != 0) {
    const int up = (pl.H + 3) & ~3;
    if (up <= N && (size_t)up * (N + 2 * kPad) * BT <= 17408 &&
        (size_t)up * N * BT <= (size_t)4 * kPF * kFT)
      pl.H = up;
    else if (pl.H >= 4)
      pl.H &= ~3;
  }
  const int nbands = (N + pl.H - 1) / pl.H;
  const int slots = (tune.fwd_slots > 0 ? tune.fwd_slots : 2) * num_cu();
  int want = std::max(1, std::min(slots / (pl.n_chunks * pl.n_tiles), nbands));
  pl.G = (nbands + want - 1) / want;
  pl.n_groups = (nbands + pl.G - 1) / pl.G;
  pl.n_ord = 0;
  return pl;
}

// Rows a ray crosses inside the padded image (the band kernel's per-ray row
// range, as a count).
static double ray_rows(const AngleGeom& g, int N, int t) {
  const double lo_p = kPad - 1.5, hi_p = N + kPad + 0.5;
  if (g.f_n1 == 0.0) {
    const double p0 = t * g.f_inv + g.f_c0;
    return (p0 < lo_p || p0 > hi_p) ? 0.0 : (double)N;
  }
  const double ma = g.f_qa + t * g.f_qs, mb = g.f_qb + t * g.f_qs;
  const double lo = std::max(0.0, std::ceil(std::min(ma, mb)));
  const double hi = std::min((double)(N - 1), std::floor(std::max(ma, mb)));
  return hi >= lo ? hi - lo + 1.0 : 0.0;
}

// Workgroup order that evens out the CUs' work.  A launch's workgroups are
// spread over the eight XCDs by position (xcd_position); within an XCD the
// first round of positions takes one CU each and the second round the
// second slot of the same CUs, in the same order.  Each chunk's work (rows
// summed over its rays, estimated from 32 sampled rays) is the same for
// every band group, so the first round takes the heaviest chunks of each
// position's tile-group and the second round gives the lightest remaining
// chunk to the position whose CU partner is heaviest; later rounds take the
// heaviest first.  Every tile-group still holds each chunk once, so only the
// schedule changes, never a result.
static void order_chunks_compute(FwdPlan& pl, const AngleGeom* h_geom, int N, int R) {
  const int total = pl.n_groups * pl.n_chunks * pl.n_tiles;
  const int ncu = num_cu();
  if (total > kMaxOrd || pl.n_chunks > 255 || ncu % 8 != 0 || total <= ncu / 8) return;
  std::vector<double> work(pl.n_chunks);
  const int nrc = (pl.n_row * R + pl.per - 1) / pl.per;
  for (int c = 0; c < pl.n_chunks; ++c) {
    const bool colm = c >= nrc;
    const int eg = colm ? pl.n_row : 0, ng = colm ? pl.n - pl.n_row : pl.n_row;
    const int i0 = (colm ? c - nrc : c) * pl.per;
    const int i1 = std::min(ng * R, i0 + pl.per);
    const int il = 1 << pl.il_lg, full = (ng >> pl.il_lg) << pl.il_lg;
    double sum = 0.0;
    constexpr int S = 32;
    for (int k = 0; k < S; ++k) {
      const int j = i0 + (int)((k + 0.5) * (i1 - i0) / S);
      int e, t;
      if (j < full * R) {
        const int m = j / (il * R), rem = j - m * il * R;
        e = il * m + (rem & (il - 1));
        t = rem >> pl.il_lg;
      } else {
        const int j2 = j - full * R, kk = ng - full;
        e = full + j2 % kk;
        t = j2 / kk;
      }
      sum += ray_rows(h_geom[pl.id[eg + e]], N, t);
    }
    work[c] = sum * (i1 - i0) / S;
  }
  std::vector<int> byw(pl.n_chunks);
  for (int c = 0; c < pl.n_chunks; ++c) byw[c] = c;
  std::stable_sort(byw.begin(), byw.end(), [&](int a, int b) { return work[a] > work[b]; });
  const int n_tg = pl.n_groups * pl.n_tiles;
  std::vector<int> head(n_tg, 0), tail(n_tg, pl.n_chunks);   // unused part of byw per tile-group
  const int cux = ncu / 8;
  const int per_xcd = (total + 7) / 8;
  std::vector<int> cu_work(cux);
  std::vector<int> round1;
  for (int x = 0; x < 8; ++x) {
    const int base = x * per_xcd;
    for (int p = 0; p < per_xcd; ++p) {
      const int pos = base + p;
      if (pos >= total) break;
      const int tg = pos / pl.n_chunks;
      if (p < cux) {
        const int c = byw[head[tg]++];
        pl.corder[pos] = (unsigned char)c;
        cu_work[p] = (int)work[c];
      } else if (p < 2 * cux) {
        round1.push_back(p);
      } else {
        pl.corder[pos] = (unsigned char)byw[head[tg]++];
      }
      if (p + 1 == std::min(per_xcd, 2 * cux) || pos + 1 == total) {
        // second round: heaviest partners first, each takes its tile-group's lightest chunk
        std::stable_sort(round1.begin(), round1.end(),
                         [&](int a, int b) { return cu_work[a - cux] > cu_work[b - cux]; });
        for (int q : round1) {
          const int tq = (base + q) / pl.n_chunks;
          pl.corder[base + q] = (unsigned char)byw[--tail[tq]];
        }
        round1.clear();
      }
    }
  }
  // each tile-group must hold every chunk exactly once; else keep the plain order
  std::vector<unsigned char> seen((size_t)n_tg * pl.n_chunks, 0);
  for (int pos = 0; pos < total; ++pos) {
    const int c = pl.corder[pos];
    if (c >= pl.n_chunks || seen[(size_t)(pos / pl.n_chunks) * pl.n_chunks + c]++) return;
  }
  pl.n_ord = total;
}

// The order of the last few plans, so a CG solve (one plan per window,
// launched every iteration) computes it once.  An entry matches on the
// plan's shape and angle order and on the geometry table's address; the
// order it returns is a permutation of this shape's chunks in any case.
struct OrderEntry {
  const AngleGeom* geom = nullptr;
  int N = 0, R = 0, n = 0, n_row = 0, per = 0, il_lg = 0, n_chunks = 0, total = 0;
  short id[kMaxList];
  int n_ord = 0;
  unsigned char corder[kMaxOrd];
};
static std::mutex g_ord_mu;
static OrderEntry g_ord[8];
static int g_ord_next = 0;

static void order_chunks(FwdPlan& pl, const AngleGeom* h_geom, int N, int R) {
  const int total = pl.n_groups * pl.n_chunks * pl.n_tiles;
  auto same = [&](const OrderEntry& o) {
    return o.geom == h_geom && o.N == N && o.R == R && o.n == pl.n && o.n_row == pl.n_row &&
           o.per == pl.per && o.il_lg == pl.il_lg && o.n_chunks == pl.n_chunks &&
           o.total == total && std::memcmp(o.id, pl.id, sizeof(short) * pl.n) == 0;
  };
  std::lock_guard<std::mutex> lock(g_ord_mu);
  for (const OrderEntry& o : g_ord)
    if (same(o)) {
      pl.n_ord = o.n_ord;
      std::memcpy(pl.corder, o.corder, (size_t)o.n_ord);
      return;
    }
  order_chunks_compute(pl, h_geom, N, R);
  OrderEntry& o = g_ord[g_ord_next];
  g_ord_next = (g_ord_next + 1) % 8;
  o.geom = h_geom;
  o.N = N;
  o.R = R;
  o.n = pl.n;
  o.n_row = pl.n_row;
  o.per = pl.per;
  o.il_lg = pl.il_lg;
  o.n_chunks = pl.n_chunks;
  o.total = total;
  std::memcpy(o.id, pl.id, sizeof(short) * pl.n);
  o.n_ord = pl.n_ord;
  std::memcpy(o.corder, pl.corder, (size_t)pl.n_ord);
}

int forward_max_items(int bt) { return max_items(bt); }

size_t forward_partial_floats(const AngleGeom* h_geom, int N, int R, const AngleList& ids, int B,
                              const ProjTune& tune) {
  const FwdPlan pl = make_plan(h_geom, N, R, ids, B, tune);
  return (size_t)B * pl.n_groups * ids.n * R;
}


template <int IT, int BT, typename IMG>
static void launch_it(dim3 grid, size_t lds, hipStream_t st, const AngleGeom* geom, int N, int R,
                      const FwdPlan& pl, int B, const IMG* img, const IMG* imgT, size_t stride,
                      float* partial, const int* stop, int stop_stride) {
  hipLaunchKernelGGL((fwd_band_kernel<IT, BT, IMG>), grid, dim3(kFT), lds, st, geom, N, R, pl, B,
                     img, imgT, stride, partial, stop, stop_stride);
}

// items is one of the values item_count() returns for this BT
template <int BT, typename IMG>
static void launch_band(int items, dim3 grid, size_t lds, hipStream_t st, const AngleGeom* geom,
                        int N, int R, const FwdPlan& pl, int B, const IMG* img, const IMG* imgT,
                        size_t stride, float* partial, const int* stop, int stop_stride) {
#define SLIM_FWD_CASE(IT)                                                                 \
  case IT:                                                                              \
    launch_it<(IT <= max_items(BT) ? IT : max_items(BT)), BT, IMG>(                     \
        grid, lds, st, geom, N, R, pl, B, img, imgT, stride, partial, stop, stop_stride); \
    break;
  switch (items) {
    SLIM_FWD_CASE(1)
    SLIM_FWD_CASE(2)
    SLIM_FWD_CASE(3)
    SLIM_FWD_CASE(4)
    SLIM_FWD_CASE(5)
    SLIM_FWD_CASE(6)
    default:
      launch_it<max_items(BT), BT, IMG>(grid, lds, st, geom, N, R, pl, B, img, imgT, stride,
                                        partial, stop, stop_stride);
      break;
  }
#undef SLIM_FWD_CASE
}

template <typename IMG>
static void launch_band_bt(int BT, int items, dim3 grid, size_t lds, hipStream_t st,
                           const AngleGeom* geom, int N, int R, const FwdPlan& pl, int B,
                           const IMG* img, const IMG* imgT, size_t stride, float* partial,
                           const int* stop, int stop_stride) {
  if (BT == 4)
    launch_band<4>(items, grid, lds, st, geom, N, R, pl, B, img, imgT, stride, partial, stop,
                   stop_stride);
  else if (BT == 2)
    launch_band<2>(items, grid, lds, st, geom, N, R, pl, B, img, imgT, stride, partial, stop,
                   stop_stride);
  else
    launch_band<1>(items, grid, lds, st, geom, N, R, pl, B, img, imgT, stride, partial, stop,
                   stop_stride);
}

hipError_t launch_forward(const FwdArgs& a, hipStream_t st) {
  if (a.ids->n <= 0) return hipSuccess;
  FwdPlan pl = make_plan(a.h_geom, a.N, a.R, *a.ids, a.B, a.tune);
  order_chunks(pl, a.h_geom, a.N, a.R);
  const int BT = pl.bt;
  const bool timed = a.prof && a.prof->on;
  hipError_t e;
  if (timed && (e = a.prof->begin(K_FORWARD, st)) != hipSuccess) return e;
  const int total = pl.n_groups * pl.n_chunks * pl.n_tiles;
  const int nwg = (total + 7) / 8 * 8;
  const size_t lds = (size_t)pl.H * (a.N + 2 * kPad) * BT * sizeof(float);
  if (a.img_bf16)
    launch_band_bt(BT, pl.items, dim3(nwg), lds, st, a.geom, a.N, a.R, pl, a.B,
                   (const uint16_t*)a.img, (const uint16_t*)a.imgT, a.img_stride, a.partial,
                   a.stop, a.stop_stride);
  else
    launch_band_bt(BT, pl.items, dim3(nwg), lds, st, a.geom, a.N, a.R, pl, a.B,
                   (const float*)a.img, (const float*)a.imgT, a.img_stride, a.partial, a.stop,
                   a.stop_stride);
  if (timed && (e = a.prof->end(st)) != hipSuccess) return e;
  if (timed && (e = a.prof->begin(K_FWD_REDUCE, st)) != hipSuccess) return e;
  const int n = a.ids->n * a.R;
  const dim3 rg((n + 255) / 256, a.B);
  if (a.sub_bf16)
    hipLaunchKernelGGL(fwd_reduce_kernel<uint16_t>, rg, dim3(256), 0, st, a.geom, a.R, *a.ids,
                       pl.n_groups, a.partial, (const uint16_t*)a.sub, a.sub_stride, a.out32,
                       a.out64, a.out_stride, a.pd, a.pd_stride, a.lam, a.dots, a.dots2, a.dots_stride,
                       a.stop, a.stop_stride);
  else
    hipLaunchKernelGGL(fwd_reduce_kernel<float>, rg, dim3(256), 0, st, a.geom, a.R, *a.ids,
                       pl.n_groups, a.partial, (const float*)a.sub, a.sub_stride, a.out32, a.out64,
                       a.out_stride, a.pd, a.pd_stride, a.lam, a.dots, a.dots2, a.dots_stride, a.stop,
                       a.stop_stride);
  if ((e = hipGetLastError()) != hipSuccess) return e;
  if (timed && (e = a.prof->end(st)) != hipSuccess) return e;
  return hipSuccess;
}

int back_num_workgroups(int N) { return ((N + kBW - 1) / kBW) * ((N + kBH - 1) / kBH); }

template <typename VT, int BT, int RB>
static void launch_back_t(const BackArgs& a, const VT* v, dim3 grid, hipStream_t st) {
  hipLaunchKernelGGL((back_kernel<VT, BT, RB>), grid, dim3(256), 0, st, a.geom, a.N, a.R, *a.ids, a.B, v,
                     a.v_stride, a.out, a.x, a.xT, a.x_true, a.img_stride, a.partials, a.mode,
                     a.stop, a.stop_stride, a.xs, a.xsT, a.shrink);
}

template <typename VT>
static void launch_back_bt(const BackArgs& a, const VT* v, hipStream_t st) {
  const int BT = a.tune.back_bt > 0 ? std::min(a.tune.back_bt, slice_tile(a.B)) : slice_tile(a.B);
  // Without the update (mode 0): tiles of two row blocks (32 x 64), so each
  // lane's per-angle set-up serves 8 pixels and each workgroup's staged
  // segments twice the pixels.  Every mode-0 launch (any slice tile, and the
  // grouped one) uses them, so a slice's result does not depend on the
  // launch it is in.
  const int RB = a.mode == 0 ? 2 : 1;
  dim3 grid((a.N + kBW - 1) / kBW, (a.N + RB * kBH - 1) / (RB * kBH), (a.B + BT - 1) / BT);
  if (RB == 2) {
    if (BT == 4)
      launch_back_t<VT, 4, 2>(a, v, grid, st);
    else if (BT == 2)
      launch_back_t<VT, 2, 2>(a, v, grid, st);
    else
      launch_back_t<VT, 1, 2>(a, v, grid, st);
  } else {
    if (BT == 4)
      launch_back_t<VT, 4, 1>(a, v, grid, st);
    else if (BT == 2)
      launch_back_t<VT, 2, 1>(a, v, grid, st);
    else
      launch_back_t<VT, 1, 1>(a, v, grid, st);
  }
}

hipError_t launch_back(const BackArgs& a, hipStream_t st) {
  if (a.v64)
    launch_back_bt(a, a.v64, st);
  else
    launch_back_bt(a, a.v32, st);
  return hipGetLastError();
}

static size_t align256(size_t b) { return (b + 255) & ~size_t(255); }

size_t grouped_desc_bytes(int n) {
  return align256(n * sizeof(FwdGroupDesc)) + align256(n * sizeof(RedGroupDesc)) +
         align256(n * sizeof(BackGroupDesc));
}

hipError_t grouped_prepare(const FwdArgs* const* fa, const BackArgs* const* ba, int n,
                           void* host_desc, GroupShape* shape) {
  if (n < 1) return hipErrorInvalidValue;
  char* base = static_cast<char*>(host_desc);
  FwdGroupDesc* fd = reinterpret_cast<FwdGroupDesc*>(base);
  RedGroupDesc* rd = reinterpret_cast<RedGroupDesc*>(base + align256(n * sizeof(FwdGroupDesc)));
  BackGroupDesc* bd = reinterpret_cast<BackGroupDesc*>(
      base + align256(n * sizeof(FwdGroupDesc)) + align256(n * sizeof(RedGroupDesc)));
  GroupShape sh;
  sh.n = n;
  sh.back_bt = 4;
  for (int g = 0; g < n; ++g) {
    const BackArgs& b = *ba[g];
    const int bt = b.tune.back_bt > 0 ? std::min(b.tune.back_bt, slice_tile(b.B)) : slice_tile(b.B);
    sh.back_bt = std::min(sh.back_bt, bt);
  }
  for (int g = 0; g < n; ++g) {
    const FwdArgs& a = *fa[g];
    const BackArgs& b = *ba[g];
    if (a.img_bf16 || a.sub || !a.pd || a.out32 || b.v32 || b.mode != 0)
      return hipErrorInvalidValue;  // only the CG products are grouped
    const FwdPlan pl = make_plan(a.h_geom, a.N, a.R, *a.ids, a.B, a.tune);
    FwdGroupDesc& f = fd[g];
    f.pl = pl;
    f.geom = a.geom;
    f.img = static_cast<const float*>(a.img);
    f.imgT = static_cast<const float*>(a.imgT);
    f.partial = a.partial;
    f.stop = a.stop;
    f.img_stride = a.img_stride;
    f.N = a.N;
    f.R = a.R;
    f.B = a.B;
    f.stop_stride = a.stop_stride;
    f.total = pl.n_groups * pl.n_chunks * pl.n_tiles;
    f.per = (f.total + 7) / 8;
    f.start = sh.band_grid / 8;
    sh.band_grid += 8 * f.per;
    f.bt = pl.bt;
    f.items = pl.items;
    // the (slice tile, rays per lane) pairs the grouped band kernel holds
    const bool known = (pl.bt == 1 && ((pl.items >= 1 && pl.items <= 6) || pl.items == 8)) ||
                       (pl.bt == 2 && pl.items >= 1 && pl.items <= 6) ||
                       (pl.bt == 4 && pl.items >= 1 && pl.items <= 3);
    if (!known) return hipErrorInvalidValue;
    sh.band_total += f.total;
    sh.band_lds = std::max(sh.band_lds, (size_t)pl.H * (a.N + 2 * kPad) * pl.bt * sizeof(float));
    RedGroupDesc& r = rd[g];
    r.ids = *a.ids;
    r.geom = a.geom;
    r.partial = a.partial;
    r.out64 = a.out64;
    r.pd = a.pd;
    r.dots = a.dots;
    r.dots2 = a.dots2;
    r.stop = a.stop;
    r.out_stride = a.out_stride;
    r.pd_stride = a.pd_stride;
    r.dots_stride = a.dots_stride;
    r.lam = a.lam;
    r.R = a.R;
    r.n_groups = pl.n_groups;
    r.gx = (a.ids->n * a.R + 255) / 256;
    r.stop_stride = a.stop_stride;
    r.start = sh.red_total;
    sh.red_total += r.gx * a.B;
    BackGroupDesc& k = bd[g];
    k.ids = *b.ids;
    k.geom = b.geom;
    k.v = b.v64;
    k.out = b.out;
    k.xT = b.xT;
    k.stop = b.stop;
    k.v_stride = b.v_stride;
    k.img_stride = b.img_stride;
    k.N = b.N;
    k.R = b.R;
    k.B = b.B;
    k.gx = (b.N + kBW - 1) / kBW;
    k.gy = (b.N + 2 * kBH - 1) / (2 * kBH);   // mode 0: tiles of two row blocks
    k.stop_stride = b.stop_stride;
    k.start = sh.back_total;
    sh.back_total += k.gx * k.gy * ((b.B + sh.back_bt - 1) / sh.back_bt);
  }
  *shape = sh;
  return hipSuccess;
}

hipError_t launch_back_grouped(const void* dev_desc, const GroupShape& sh, hipStream_t st) {
  const char* base = static_cast<const char*>(dev_desc);
  const BackGroupDesc* bd = reinterpret_cast<const BackGroupDesc*>(
      base + align256(sh.n * sizeof(FwdGroupDesc)) + align256(sh.n * sizeof(RedGroupDesc)));
  if (sh.back_total <= 0) return hipSuccess;
  if (sh.back_bt == 4)
    hipLaunchKernelGGL(back_grouped<4>, dim3(sh.back_total), dim3(256), 0, st, bd, sh.n);
  else if (sh.back_bt == 2)
    hipLaunchKernelGGL(back_grouped<2>, dim3(sh.back_total), dim3(256), 0, st, bd, sh.n);
  else
    hipLaunchKernelGGL(back_grouped<1>, dim3(sh.back_total), dim3(256), 0, st, bd, sh.n);
  return hipGetLastError();
}

hipError_t launch_forward_grouped(const void* dev_desc, const GroupShape& sh, hipStream_t st) {
  const char* base = static_cast<const char*>(dev_desc);
  const FwdGroupDesc* fd = reinterpret_cast<const FwdGroupDesc*>(base);
  const RedGroupDesc* rd =
      reinterpret_cast<const RedGroupDesc*>(base + align256(sh.n * sizeof(FwdGroupDesc)));
  if (sh.band_total > 0)
    hipLaunchKernelGGL(fwd_band_grouped, dim3(sh.band_grid), dim3(kFT), sh.band_lds, st, fd, sh.n);
  if (sh.red_total > 0)
    hipLaunchKernelGGL(fwd_reduce_grouped, dim3(sh.red_total), dim3(256), 0, st, rd, sh.n);
  return hipGetLastError();
}

hipError_t launch_reduce3(const double* partials, int n, int B, double* out, hipStream_t st) {
  hipLaunchKernelGGL(reduce3_kernel, dim3(B), dim3(256), 0, st, partials, n, out);
  return hipGetLastError();
}

hipError_t launch_transpose(const float* src, float* dst, int N, int B, size_t stride,
                            uint16_t* bs, uint16_t* bsT, hipStream_t st) {
  const int t = (N + kTile - 1) / kTile;
  hipLaunchKernelGGL(transpose_kernel, dim3(t, t, B), dim3(256), 0, st, src, dst, N, stride, bs,
                     bsT);
  return hipGetLastError();
}

hipError_t launch_gather_rows(const void* b, int b_bf16, int n_angles, int R, int B,
                              const AngleList& ids, float* out, hipStream_t st) {
  const dim3 grid((R + 255) / 256, ids.n, B);
  if (b_bf16)
    hipLaunchKernelGGL(gather_rows_kernel<uint16_t>, grid, dim3(256), 0, st, (const uint16_t*)b,
                       n_angles, R, ids, out);
  else
    hipLaunchKernelGGL(gather_rows_kernel<float>, grid, dim3(256), 0, st, (const float*)b,
                       n_angles, R, ids, out);
  return hipGetLastError();
}

}  // namespace slim
