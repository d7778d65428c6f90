// Matrix-free 3D parallel-beam projectors (Joseph's method along the major
// axis) and the float64 CG kernels of the 3D slimLS path, for gfx950.
//
// Forward (ray-driven): the volume is read in a padded layout stored with
// the direction's major axis m slowest, so every plane x_m = const a ray
// crosses is a contiguous block of rows along the axis a, each starting on a
// 16-byte boundary.  A workgroup owns a 16 x 16 tile of detector pixels of
// one direction and one of kSeg segments of the planes, and walks the planes
// its rays cross four at a time: the box of voxels around the tile's
// crossing points in each plane (at most 32 x 32: a detector step moves the
// crossing point by at most 2 voxels along a and along b) is staged in LDS
// with 16-byte loads, zeros outside the volume; every lane then advances its
// crossing point in 32.32 fixed point (one 64-bit add per plane and axis) and
// interpolates bilinearly between the four voxel centres around it.  Ray sums
// run in float32 over 32 planes and accumulate in float64; a second kernel
// adds the segments' sums in a fixed order and applies h/|w_m|, the data and
// the CG tail.
//
// Back (voxel-driven gather, the exact adjoint): a workgroup owns a tile of
// 16 x 16 x 8 voxels, a lane a column of 8 along z; per direction it stages
// the detector window its tile projects onto (at most 27 x 28 of the
// 32 x 32 LDS pixels, scaled by h/|w_m|) and every voxel evaluates the
// closed-form weights of the candidate rays around its own ray (2 or 3
// detector columns times 2 or 3 rows, by the direction): the crossing-point
// displacement is linear in the detector offset (DirGeom), and a weight is
// the product of two tents.
#include "slim3d_internal.h"

namespace slim {
namespace {

constexpr int kRT = 16;                   // forward ray tile (t and q)
constexpr int kVX = 16, kVY = 16, kVZ = 8;  // back-projector voxel tile (a lane: kVZ along z)
constexpr int kFP = 32;                     // staged detector window side
constexpr int kFS = kFP + 1;                // its LDS row stride (odd: rows fall in distinct banks)
constexpr int kFlush = 32;                // planes per float32 partial sum
constexpr double kTwo32 = 4294967296.0;
constexpr float kInv32 = 2.3283064365386963e-10f;  // 2^-32

// Planes k with -1 < f0 + k s < N (the crossing index f along one axis),
// intersected into [lo, hi] (real bounds; callers round outwards).
__device__ __forceinline__ void plane_range(double f0, double s, int N, double& lo, double& hi) {
  if (s > 0.0) {
    lo = fmax(lo, (-1.0 - f0) / s);
    hi = fmin(hi, ((double)N - f0) / s);
  } else if (s < 0.0) {
    lo = fmax(lo, ((double)N - f0) / s);
    hi = fmin(hi, (-1.0 - f0) / s);
  } else if (!(f0 > -1.0 && f0 < (double)N)) {
    hi = -2.0;
  }
}

__device__ __forceinline__ float unit_clamp(float v) { return __builtin_amdgcn_fmed3f(v, 0.f, 1.f); }

__device__ __forceinline__ double block_sum(double v, double* sh) {
  for (int o = 32; o > 0; o >>= 1) v += __shfl_down(v, o, 64);
  if ((threadIdx.x & 63) == 0) sh[threadIdx.x >> 6] = v;
  __syncthreads();
  const double s = sh[0] + sh[1] + sh[2] + sh[3];
  __syncthreads();
  return s;
}

// Index of voxel (z k, y i, x j) in the padded volume stored with axis m
// slowest: plane k_m, then axis b, then axis a fastest (a < b the other two
// axes), each row of N voxels preceded by kPad zeros and padded with zeros to
// the pitch lay_pitch(N), a multiple of four; a plane crossed by the rays of
// a direction with major axis m is one contiguous block of N rows.
__device__ __forceinline__ size_t lay_index(int m, int N, int P, int k, int i, int j) {
  if (m == 2) return ((size_t)k * N + i) * P + j + kPad;
  if (m == 1) return ((size_t)i * N + k) * P + j + kPad;
  return ((size_t)j * N + k) * P + i + kPad;
}

// Forward: the planes along m are cut into kSeg segments, one workgroup per
// (ray tile, direction, segment), each writing its rays' partial sums; a
// second kernel adds the segments in a fixed order.
constexpr int kSeg = 8;
constexpr int kSlab = 4;            // planes staged per pass
constexpr int kBA = 40, kBB = 34;   // staged box per plane: voxels along a, rows along b

constexpr int kStage = (kSlab * kBB * kBA / 4 + 255) / 256;   // 16-byte loads per lane per slab

__global__ __launch_bounds__(256) void fwd3_kernel(
    const DirGeom* __restrict__ geom, DirList ids, int N, int n, const float* __restrict__ lay0,
    const float* __restrict__ lay1, const float* __restrict__ lay2, double* __restrict__ part,
    size_t part_stride, const int* __restrict__ ctl) {
  if (ctl && ctl[kCtlDone]) return;
  __shared__ __align__(16) float box[kSlab * kBB * kBA];
  __shared__ int kr[8];
  // XCD-aware numbering: consecutive positions (neighbouring tiles, whose
  // boxes overlap) run on one XCD and share its L2
  const int gt = (n + kRT - 1) / kRT;
  const int per_xcd = gridDim.x >> 3;
  const int pos = (blockIdx.x & 7) * per_xcd + (blockIdx.x >> 3);
  if (pos >= gt * gt * kSeg * ids.n) return;
  const int tt = pos % gt, tq = (pos / gt) % gt, ss = pos / (gt * gt);
  const int slot = ss / kSeg, seg = ss - slot * kSeg;
  const DirGeom G = geom[ids.id[slot]];
  const float* __restrict__ vol = G.m == 0 ? lay0 : (G.m == 1 ? lay1 : lay2);
  const int P = lay_pitch(N);
  const int tid = threadIdx.x;
  const int t = tt * kRT + (tid & (kRT - 1));
  const int q = tq * kRT + (tid / kRT);
  const bool live = t < n && q < n;
  const double hN = 0.5 * (N - 1), hn = 0.5 * (n - 1);
  const double fa0 = hN + (t - hn) * G.La[0] + (q - hn) * G.La[1] - hN * G.sa;
  const double fb0 = hN + (t - hn) * G.Lb[0] + (q - hn) * G.Lb[1] - hN * G.sb;
  // the crossing points of the tile's rays (live or not) in plane k lie in
  // [amin0 + k sa, amin0 + k sa + aspan] along a (b likewise): the tile's
  // corners bound them, the crossing point being linear in (t, q)
  const double tc = tt * kRT - hn, qc = tq * kRT - hn;
  const double amin0 = hN + tc * G.La[0] + qc * G.La[1] - hN * G.sa +
                       fmin(0.0, (kRT - 1) * G.La[0]) + fmin(0.0, (kRT - 1) * G.La[1]);
  const double bmin0 = hN + tc * G.Lb[0] + qc * G.Lb[1] - hN * G.sb +
                       fmin(0.0, (kRT - 1) * G.Lb[0]) + fmin(0.0, (kRT - 1) * G.Lb[1]);
  const double aspan = (kRT - 1) * (fabs(G.La[0]) + fabs(G.La[1]));   // <= 30
  const double bspan = (kRT - 1) * (fabs(G.Lb[0]) + fabs(G.Lb[1]));
  // staged per plane: rows floor(bmin) - 1 .. floor(bmin) + ceil(bspan) + 2
  // and voxels from floor(amin) - 1 rounded down to a multiple of four to
  // floor(amin) + ceil(aspan) + 2, one voxel of slack on either side for
  // rounding between the lanes' crossing points and the box's
  const int nrow = min(kBB, (int)ceil(bspan) + 4);
  const int nvec = min(kBA / 4, ((int)ceil(aspan) + 7 + 3) / 4);
  // the ray's planes (-1 < f < N on both axes) within this segment
  const int s0 = seg * N / kSeg, s1 = (seg + 1) * N / kSeg - 1;
  double lo = (double)s0, hi = (double)s1;
  plane_range(fa0, G.sa, N, lo, hi);
  plane_range(fb0, G.sb, N, lo, hi);
  int k0 = live ? (int)fmin((double)N, fmax((double)s0, floor(lo))) : N;
  int k1 = live ? (int)fmax(-1.0, fmin((double)s1, ceil(hi))) : -1;
  if (k0 > k1) {
    k0 = N;
    k1 = -1;
  }
  // the workgroup walks the union of its rays' plane ranges (a lane outside
  // its own range finds its crossing point outside the volume: zeros)
  for (int o = 32; o > 0; o >>= 1) {
    k0 = min(k0, __shfl_xor(k0, o, 64));
    k1 = max(k1, __shfl_xor(k1, o, 64));
  }
  if ((tid & 63) == 0) {
    kr[tid >> 6] = k0;
    kr[4 + (tid >> 6)] = k1;
  }
  __syncthreads();
  const int K0 = min(min(kr[0], kr[1]), min(kr[2], kr[3]));
  const int K1 = max(max(kr[4], kr[5]), max(kr[6], kr[7]));
  double sum = 0.0;
  if (K0 <= K1) {
    const size_t sm = (size_t)N * P;
    // crossing points (lanes) and box corners in 32.32 fixed point from K0,
    // all advanced by the same per-plane steps
    const int64_t Sa = llrint(G.sa * kTwo32), Sb = llrint(G.sb * kTwo32);
    int64_t Fa = llrint((fa0 + K0 * G.sa) * kTwo32), Fb = llrint((fb0 + K0 * G.sb) * kTwo32);
    const int64_t Ma = llrint((amin0 + K0 * G.sa) * kTwo32), Mb = llrint((bmin0 + K0 * G.sb) * kTwo32);
    const int per = nrow * nvec;
    const float inv_per = 1.0f / (float)per, inv_nvec = 1.0f / (float)nvec;
    // slab staging in two halves: the loads of slab k + kSlab are in flight
    // while slab k is interpolated from LDS
    float4 pre[kStage];
    int off[kStage];
    auto load_slab = [&](int k) {
      const int np = min(kSlab, K1 - k + 1);
#pragma unroll
      for (int u = 0; u < kStage; ++u) {
        const int e = tid + 256 * u;
        pre[u] = make_float4(0.f, 0.f, 0.f, 0.f);
        off[u] = -1;
        if (e < np * per) {
          // exact: the quotients' fractional parts stay >= 0.5 / per from integers
          const int pl = (int)(((float)e + 0.5f) * inv_per);
          const int r = e - pl * per;
          const int row = (int)(((float)r + 0.5f) * inv_nvec);
          const int c = r - row * nvec;
          const int64_t dk = k + pl - K0;
          const int A0 = ((int)((Ma + dk * Sa) >> 32) - 1) & ~3;
          const int b = (int)((Mb + dk * Sb) >> 32) - 1 + row;
          const int as = A0 + 4 * c + kPad;
          off[u] = (pl * kBB + row) * kBA + 4 * c;
          if ((unsigned)b < (unsigned)N && as >= 0 && as + 4 <= P)
            pre[u] = *reinterpret_cast<const float4*>(vol + ((size_t)(k + pl) * sm + (size_t)b * P + as));
        }
      }
    };
    load_slab(K0);
    float acc = 0.f;
    int cnt = 0;
    for (int k = K0; k <= K1; k += kSlab) {
      const int np = min(kSlab, K1 - k + 1);
      __syncthreads();  // the previous slab's reads are done
#pragma unroll
      for (int u = 0; u < kStage; ++u)
        if (off[u] >= 0) *reinterpret_cast<float4*>(box + off[u]) = pre[u];
      __syncthreads();
      if (k + kSlab <= K1) load_slab(k + kSlab);
#pragma unroll
      for (int pl = 0; pl < kSlab; ++pl) {
        if (pl < np) {
          const int64_t dk = k + pl - K0;
          const int A0 = ((int)((Ma + dk * Sa) >> 32) - 1) & ~3;
          const int B0 = (int)((Mb + dk * Sb) >> 32) - 1;
          const int ia = (int)(Fa >> 32), ib = (int)(Fb >> 32);
          const float fa = (float)(uint32_t)Fa * kInv32, fb = (float)(uint32_t)Fb * kInv32;
          // never clamped for a ray of the tile (see the box bounds above)
          const int la = min(max(ia - A0, 0), kBA - 2), lb = min(max(ib - B0, 0), kBB - 2);
          const float* bx = box + (pl * kBB + lb) * kBA + la;
          const float v00 = bx[0], v10 = bx[1], v01 = bx[kBA], v11 = bx[kBA + 1];
          const float lo_b = fmaf(fa, v10 - v00, v00);
          const float hi_b = fmaf(fa, v11 - v01, v01);
          acc += fmaf(fb, hi_b - lo_b, lo_b);
          Fa += Sa;
          Fb += Sb;
          if (++cnt == kFlush) {
            sum += (double)acc;
            acc = 0.f;
            cnt = 0;
          }
        }
      }
    }
    sum += (double)acc;
  }
  if (live) part[seg * part_stride + ((size_t)slot * n + q) * n + t] = sum;
}

// out[s][q][t] = (h/|w_m|) sum_segments part - sub for every ray (fixed
// order); optional CG tail q = out + lam pd with per-workgroup partial dots.
__global__ __launch_bounds__(256) void fwd3_reduce_kernel(
    const DirGeom* __restrict__ geom, DirList ids, int n, const double* __restrict__ part,
    size_t part_stride, const float* __restrict__ sub, float* __restrict__ out32,
    double* __restrict__ out64, const double* __restrict__ pd, double lam,
    double* __restrict__ dots, const int* __restrict__ ctl) {
  if (ctl && ctl[kCtlDone]) return;
  __shared__ double sh[4];
  const size_t nn = (size_t)n * n;
  const size_t o = (size_t)blockIdx.x * 256 + threadIdx.x;
  const size_t tot = nn * ids.n;
  double d = 0.0;
  if (o < tot) {
    const int slot = (int)(o / nn);
    double v = 0.0;
#pragma unroll
    for (int sg = 0; sg < kSeg; ++sg) v += part[sg * part_stride + o];
    v *= geom[ids.id[slot]].scale;
    if (sub) v -= (double)sub[(size_t)ids.id[slot] * nn + (o - slot * nn)];
    if (pd) {
      const double pv = pd[o];
      v = fma(lam, pv, v);
      d = pv * v;
    }
    if (out64) out64[o] = v;
    if (out32) out32[o] = (float)v;
  }
  if (dots) {
    const double s = block_sum(d, sh);
    if (threadIdx.x == 0) dots[blockIdx.x] = s;
  }
}

// dst = the standard-layout volume src in the padded layout of major axis m
// (lay_index; the pads are never written).  m = 1, 2: rows along x move
// whole, a wave per row.
__global__ __launch_bounds__(256) void relayout3_rows_kernel(const float* __restrict__ src,
                                                             float* __restrict__ dst, int N, int m) {
  const int P = lay_pitch(N);
  const int i = blockIdx.x;
  const int k = blockIdx.y * 4 + threadIdx.x / 64;
  if (k >= N) return;
  const float* __restrict__ s = src + ((size_t)k * N + i) * N;
  float* __restrict__ d = dst + lay_index(m, N, P, k, i, 0);
  for (int j = threadIdx.x & 63; j < N; j += 64) d[j] = s[j];
}

// m = 0 ([x][z][y]): every z plane is transposed through a padded 64 x 64
// LDS tile, both sides in 256-byte rows.
__global__ __launch_bounds__(256) void relayout3_x_kernel(const float* __restrict__ src,
                                                          float* __restrict__ dst, int N) {
  __shared__ float tile[64 * 65];
  const int P = lay_pitch(N);
  const int j0 = blockIdx.x * 64, i0 = blockIdx.y * 64, k = blockIdx.z;
  const int l = threadIdx.x & 63, w = threadIdx.x / 64;
  for (int r = w; r < 64; r += 4) {
    const int i = i0 + r, j = j0 + l;
    if (i < N && j < N) tile[r * 65 + l] = src[((size_t)k * N + i) * N + j];
  }
  __syncthreads();
  for (int r = w; r < 64; r += 4) {
    const int j = j0 + r, i = i0 + l;
    if (i < N && j < N) dst[lay_index(0, N, P, k, i, j)] = tile[l * 65 + r];
  }
}

// Back-projection: a workgroup owns kVX x kVY voxels (x, y) of kVZ
// consecutive z planes, a lane one (x, y) column of kVZ voxels.  Per
// direction the detector window of the whole tile is staged in LDS (scaled
// by h/|w_m|); every voxel then visits its candidate rays (see above).
template <typename VT>
__global__ __launch_bounds__(256) void back3_kernel(
    const DirGeom* __restrict__ geom, DirList ids, int N, int n, const VT* __restrict__ v,
    float* __restrict__ out, float* __restrict__ out0, float* __restrict__ out1,
    float* __restrict__ out2, float* __restrict__ x, const float* __restrict__ x_true,
    double* __restrict__ partials, int mode, const int* __restrict__ ctl) {
  if (ctl && ctl[kCtlDone]) return;
  __shared__ float sv[kFP * kFS];
  __shared__ float tr[kVZ * kVY * (kVX + 1)];   // the tile, for the x-slowest layout
  __shared__ double sh[4];
  const int tid = threadIdx.x;
  const int jl = tid & (kVX - 1), il = tid / kVX;
  const int j = blockIdx.x * kVX + jl, i = blockIdx.y * kVY + il, kb = blockIdx.z * kVZ;
  const int nk = min(kVZ, N - kb);
  const bool ok = i < N && j < N;
  const double hN = 0.5 * (N - 1), hn = 0.5 * (n - 1);
  const double cx = j - hN, cy = i - hN, cz = kb - hN;                // centre / h
  const double tx0 = blockIdx.x * kVX - hN, ty0 = blockIdx.y * kVY - hN;
  float acc[kVZ];
#pragma unroll
  for (int c = 0; c < kVZ; ++c) acc[c] = 0.f;
  for (int s = 0; s < ids.n; ++s) {
    const DirGeom G = geom[ids.id[s]];
    // detector window of the tile: its voxels' projections, floor - 1 .. floor + 2,
    // with one more pixel on the low side for rounding between fu and umin
    // (at most 15 sqrt 2 + 5 < 27 pixels along u, sqrt(15^2 + 15^2 + 7^2) + 5 < 28 along v)
    const double ub = tx0 * G.eu[0] + ty0 * G.eu[1] + cz * G.eu[2] + hn;
    const double vb = tx0 * G.ev[0] + ty0 * G.ev[1] + cz * G.ev[2] + hn;
    const double umin = ub + fmin(0.0, (kVX - 1) * G.eu[0]) + fmin(0.0, (kVY - 1) * G.eu[1]) +
                        fmin(0.0, (kVZ - 1) * G.eu[2]);
    const double vmin = vb + fmin(0.0, (kVX - 1) * G.ev[0]) + fmin(0.0, (kVY - 1) * G.ev[1]) +
                        fmin(0.0, (kVZ - 1) * G.ev[2]);
    const int t0 = (int)floor(umin) - 2, q0 = (int)floor(vmin) - 2;
    const float sc = (float)G.scale;
    const VT* vs = v + (size_t)s * n * n;
    __syncthreads();  // the previous direction's reads are done
    for (int e = tid; e < kFP * kFP; e += 256) {
      const int tq = q0 + e / kFP, tt = t0 + e % kFP;
      float val = 0.f;
      if ((unsigned)tq < (unsigned)n && (unsigned)tt < (unsigned)n)
        val = (float)vs[(size_t)tq * n + tt] * sc;
      sv[(e / kFP) * kFS + e % kFP] = val;
    }
    __syncthreads();
    if (ok) {
      // candidate rays: |du| < wu = |e_u[a]| + |e_u[b]| (dv likewise), i.e.
      // the integers of the open interval (fu - wu, fu + wu), at most
      // ceil(2 wu) <= 3 of them (2 x 2 for a direction along an axis)
      const double wu = G.wu, wv = G.wv;
      const int nt = (int)ceil(2.0 * wu), nq = (int)ceil(2.0 * wv);
      // e_u has no z component, so a column's voxels share fu: its detector
      // columns, their offsets du and the du terms of both tents are the
      // column's (fu is evaluated as cx e_u[0] + cy e_u[1] + hn)
      const double fu = cx * G.eu[0] + cy * G.eu[1] + hn;
      const double fv_xy = cx * G.ev[0] + cy * G.ev[1] + hn;
      const double tsu = floor(fu - wu) + 1.0;
      const float du0 = (float)(tsu - fu);
      // clamped so that no read leaves the window (never active for a voxel of the tile)
      const int lt = min(max((int)tsu - t0, 0), kFP - 3);
      const float la0 = (float)G.La[0], la1 = (float)G.La[1];
      const float lb0 = (float)G.Lb[0], lb1 = (float)G.Lb[1];
      float ta[3], tb[3];
#pragma unroll
      for (int ot = 0; ot < 3; ++ot) {
        ta[ot] = la0 * (du0 + (float)ot);
        tb[ot] = lb0 * (du0 + (float)ot);
      }
#pragma unroll
      for (int c = 0; c < kVZ; ++c) {
        const double fv = fma(cz + c, G.ev[2], fv_xy);
        const double tsv = floor(fv - wv) + 1.0;
        const float dv0 = (float)(tsv - fv);
        const int lq = min(max((int)tsv - q0, 0), kFP - 3);
        float a = acc[c];
#pragma unroll
        for (int oq = 0; oq < 3; ++oq) {
          if (oq < nq) {   // uniform over the workgroup (one direction)
            const float dv = dv0 + (float)oq;
            const float ra = la1 * dv, rb = lb1 * dv;
            const float* row = sv + (lq + oq) * kFS + lt;
#pragma unroll
            for (int ot = 0; ot < 3; ++ot) {
              if (ot < nt) {
                const float wa = fmaxf(1.f - fabsf(ta[ot] + ra), 0.f);
                const float wb = fmaxf(1.f - fabsf(tb[ot] + rb), 0.f);
                a = fmaf(wa * wb, row[ot], a);
              }
            }
          }
        }
        acc[c] = a;
      }
    }
  }
  if (mode == 0) {
    const int P = lay_pitch(N);
    if (ok) {
#pragma unroll
      for (int c = 0; c < kVZ; ++c) {
        if (c < nk) {
          if (out) out[((size_t)(kb + c) * N + i) * N + j] = acc[c];
          if (out2) out2[lay_index(2, N, P, kb + c, i, j)] = acc[c];
          if (out1) out1[lay_index(1, N, P, kb + c, i, j)] = acc[c];
        }
      }
    }
    if (out0) {  // rows along y: through LDS, so that a wave writes 64-byte runs
#pragma unroll
      for (int c = 0; c < kVZ; ++c) tr[(c * kVY + il) * (kVX + 1) + jl] = acc[c];
      __syncthreads();
      for (int e = tid; e < kVZ * kVY * kVX; e += 256) {
        const int il2 = e % kVY, c = (e / kVY) % kVZ, jl2 = e / (kVY * kVZ);
        const int i2 = blockIdx.y * kVY + il2, j2 = blockIdx.x * kVX + jl2;
        if (i2 < N && j2 < N && c < nk)
          out0[lay_index(0, N, P, kb + c, i2, j2)] = tr[(c * kVY + il2) * (kVX + 1) + jl2];
      }
    }
    return;
  }
  double n0 = 0.0, n1 = 0.0, n2 = 0.0;
  if (ok) {
#pragma unroll
    for (int c = 0; c < kVZ; ++c) {
      if (c < nk) {
        const size_t idx = ((size_t)(kb + c) * N + i) * N + j;
        const float xn = x[idx] - acc[c];
        x[idx] = xn;
        n0 += (double)acc[c] * acc[c];
        n1 += (double)xn * xn;
        if (x_true) {
          const double e = (double)xn - (double)x_true[idx];
          n2 += e * e;
        }
      }
    }
  }
  n0 = block_sum(n0, sh);
  n1 = block_sum(n1, sh);
  n2 = block_sum(n2, sh);
  if (tid == 0) {
    const size_t wg = ((size_t)blockIdx.z * gridDim.y + blockIdx.y) * gridDim.x + blockIdx.x;
    partials[wg * 3 + 0] = n0;
    partials[wg * 3 + 1] = n1;
    partials[wg * 3 + 2] = n2;
  }
}

// ---------------------------------------------------------------- CG
__device__ double fixed_sum(const double* __restrict__ a, int n, double* sh) {
  double v = 0.0;
  for (int k = threadIdx.x; k < n; k += 256) v += a[k];
  return block_sum(v, sh);
}

// Jacobi preconditioner of the Gram system: minv[s][q][t] = 1 / (lam +
// (A A^T) diagonal), the diagonal being the ray's squared weights summed
// over the planes it crosses; per plane the four voxels' weights are the
// products of the two axes' tents, so the squares factor into
// ((1-fa)^2 [ia inside] + fa^2 [ia+1 inside]) times the same along b.
__global__ __launch_bounds__(256) void diag3_kernel(const DirGeom* __restrict__ geom, DirList ids,
                                                    int N, int n, double lam,
                                                    double* __restrict__ minv) {
  const int slot = blockIdx.z;
  const DirGeom G = geom[ids.id[slot]];
  const int t = blockIdx.x * kRT + (threadIdx.x & (kRT - 1));
  const int q = blockIdx.y * kRT + (threadIdx.x / kRT);
  if (t >= n || q >= n) return;
  const double hN = 0.5 * (N - 1), hn = 0.5 * (n - 1);
  const double fa0 = hN + (t - hn) * G.La[0] + (q - hn) * G.La[1] - hN * G.sa;
  const double fb0 = hN + (t - hn) * G.Lb[0] + (q - hn) * G.Lb[1] - hN * G.sb;
  double lo = 0.0, hi = N - 1.0;
  plane_range(fa0, G.sa, N, lo, hi);
  plane_range(fb0, G.sb, N, lo, hi);
  const int k0 = (int)fmin((double)N, fmax(0.0, floor(lo)));
  const int k1 = (int)fmax(-1.0, fmin(N - 1.0, ceil(hi)));
  double sum = 0.0;
  if (k0 <= k1) {
    int64_t Fa = llrint((fa0 + k0 * G.sa) * kTwo32), Fb = llrint((fb0 + k0 * G.sb) * kTwo32);
    const int64_t Sa = llrint(G.sa * kTwo32), Sb = llrint(G.sb * kTwo32);
    const unsigned uN = (unsigned)N;
    float acc = 0.f;
    int cnt = 0;
    for (int k = k0; k <= k1; ++k) {
      const int ia = (int)(Fa >> 32), ib = (int)(Fb >> 32);
      const float fa = (float)(uint32_t)Fa * kInv32, fb = (float)(uint32_t)Fb * kInv32;
      const float ga = ((unsigned)ia < uN ? (1.f - fa) * (1.f - fa) : 0.f) +
                       ((unsigned)(ia + 1) < uN ? fa * fa : 0.f);
      const float gb = ((unsigned)ib < uN ? (1.f - fb) * (1.f - fb) : 0.f) +
                       ((unsigned)(ib + 1) < uN ? fb * fb : 0.f);
      acc = fmaf(ga, gb, acc);
      Fa += Sa;
      Fb += Sb;
      if (++cnt == kFlush) {
        sum += (double)acc;
        acc = 0.f;
        cnt = 0;
      }
    }
    sum += (double)acc;
  }
  minv[((size_t)slot * n + q) * n + t] = 1.0 / fma(G.scale * G.scale, sum, lam);
}

// CG init: r = e, pd = y = minv r (y = r without minv), z = 0; per-workgroup
// partial sums of r.r into parts and of r.y into parts + np.
__global__ __launch_bounds__(256) void cg3_init_kernel(const double* __restrict__ e,
                                                       const double* __restrict__ minv,
                                                       double* __restrict__ r,
                                                       double* __restrict__ pd,
                                                       double* __restrict__ z, int p,
                                                       double* __restrict__ parts) {
  __shared__ double sh[4];
  const int o = blockIdx.x * 256 + threadIdx.x;
  double d = 0.0, dy = 0.0;
  if (o < p) {
    const double v = e[o];
    const double y = minv ? minv[o] * v : v;
    r[o] = v;
    pd[o] = y;
    z[o] = 0.0;
    d = v * v;
    dy = v * y;
  }
  d = block_sum(d, sh);
  dy = block_sum(dy, sh);
  if (threadIdx.x == 0) {
    parts[blockIdx.x] = d;
    parts[gridDim.x + blockIdx.x] = dy;
  }
}

__global__ __launch_bounds__(256) void cg3_start_kernel(const double* __restrict__ parts, int np,
                                                        double* __restrict__ sc,
                                                        int* __restrict__ ctl, double tol2) {
  __shared__ double sh[4];
  const double rr = fixed_sum(parts, np, sh);
  const double ry = fixed_sum(parts + np, np, sh);
  if (threadIdx.x == 0) {
    sc[SC3_RR] = rr;
    sc[SC3_RR0] = rr;
    sc[SC3_RY] = ry;
    sc[SC3_TOL2] = tol2;
    ctl[kCtlDone] = rr > 0.0 ? 0 : 1;
    ctl[kCtlIters] = 0;
    ctl[2] = isfinite(rr) && isfinite(ry) ? 0 : 1;   // non-finite data or iterate
  }
}

__global__ __launch_bounds__(256) void cg3_alpha_kernel(const double* __restrict__ dots, int nd,
                                                        double* __restrict__ sc,
                                                        int* __restrict__ ctl) {
  if (ctl[kCtlDone]) return;
  __shared__ double sh[4];
  const double pq = fixed_sum(dots, nd, sh);
  if (threadIdx.x == 0) {
    sc[SC3_PQ] = pq;
    if (pq > 0.0 && isfinite(pq)) {
      sc[SC3_ALPHA] = sc[SC3_RY] / pq;
    } else {  // breakdown: stop with the current z
      ctl[kCtlDone] = 1;
      ctl[2] = 1;
    }
  }
}

// z += alpha pd, r -= alpha q; partial sums of r.r and r.(minv r).
__global__ __launch_bounds__(256) void cg3_update_kernel(double* __restrict__ z,
                                                         double* __restrict__ r,
                                                         const double* __restrict__ pd,
                                                         const double* __restrict__ q,
                                                         const double* __restrict__ minv, int p,
                                                         double* __restrict__ parts,
                                                         const double* __restrict__ sc,
                                                         const int* __restrict__ ctl) {
  if (ctl[kCtlDone]) return;
  __shared__ double sh[4];
  const double alpha = sc[SC3_ALPHA];
  const int o = blockIdx.x * 256 + threadIdx.x;
  double d = 0.0, dy = 0.0;
  if (o < p) {
    z[o] = fma(alpha, pd[o], z[o]);
    const double rn = fma(-alpha, q[o], r[o]);
    r[o] = rn;
    d = rn * rn;
    dy = minv ? rn * (minv[o] * rn) : d;
  }
  d = block_sum(d, sh);
  dy = block_sum(dy, sh);
  if (threadIdx.x == 0) {
    parts[blockIdx.x] = d;
    parts[gridDim.x + blockIdx.x] = dy;
  }
}

// Stop once r.r <= tol^2 e.e (r the Gram system's own residual, kept by the
// recurrence, not the preconditioned one); else beta = r.y / (r.y)_old.
__global__ __launch_bounds__(256) void cg3_rr_kernel(const double* __restrict__ parts, int np,
                                                     double* __restrict__ sc,
                                                     int* __restrict__ ctl) {
  if (ctl[kCtlDone]) return;
  __shared__ double sh[4];
  const double rr = fixed_sum(parts, np, sh);
  const double ry = fixed_sum(parts + np, np, sh);
  if (threadIdx.x == 0) {
    ctl[kCtlIters] += 1;
    if (rr <= sc[SC3_TOL2] * sc[SC3_RR0] || !isfinite(rr) || !isfinite(ry)) {
      ctl[kCtlDone] = 1;
      if (!isfinite(rr) || !isfinite(ry)) ctl[2] = 1;
    } else {
      sc[SC3_BETA] = ry / sc[SC3_RY];
    }
    sc[SC3_RR] = rr;
    sc[SC3_RY] = ry;
  }
}

__global__ __launch_bounds__(256) void cg3_pd_kernel(const double* __restrict__ r,
                                                     const double* __restrict__ minv,
                                                     double* __restrict__ pd, int p,
                                                     const double* __restrict__ sc,
                                                     const int* __restrict__ ctl) {
  if (ctl[kCtlDone]) return;
  const double beta = sc[SC3_BETA];
  const int o = blockIdx.x * 256 + threadIdx.x;
  if (o < p) pd[o] = fma(beta, pd[o], minv ? minv[o] * r[o] : r[o]);
}

}  // namespace

// ---------------------------------------------------------------- launchers
int fwd3_num_workgroups(int n, int n_ids) {
  return (int)(((size_t)n * n * n_ids + 255) / 256);
}

size_t fwd3_part_doubles(int n, int n_ids) { return (size_t)kSeg * n * n * n_ids; }

hipError_t launch_fwd3(const Fwd3Args& a, hipStream_t st) {
  if (a.ids.n <= 0) return hipSuccess;
  const int g = (a.n + kRT - 1) / kRT;
  const size_t stride = (size_t)a.n * a.n * a.ids.n;
  const int wgs = (g * g * kSeg * a.ids.n + 7) / 8 * 8;   // a multiple of the 8 XCDs
  hipLaunchKernelGGL(fwd3_kernel, dim3(wgs), dim3(256), 0, st, a.geom, a.ids, a.N,
                     a.n, a.lay[0], a.lay[1], a.lay[2], a.part, stride, a.ctl);
  hipLaunchKernelGGL(fwd3_reduce_kernel, dim3(fwd3_num_workgroups(a.n, a.ids.n)), dim3(256), 0, st,
                     a.geom, a.ids, a.n, a.part, stride, a.sub, a.out32, a.out64, a.pd, a.lam,
                     a.dots, a.ctl);
  return hipGetLastError();
}

hipError_t launch_relayout3(const float* src, float* dst, int N, int m, hipStream_t st) {
  if (m == 0)
    hipLaunchKernelGGL(relayout3_x_kernel, dim3((N + 63) / 64, (N + 63) / 64, N), dim3(256), 0, st,
                       src, dst, N);
  else
    hipLaunchKernelGGL(relayout3_rows_kernel, dim3(N, (N + 3) / 4), dim3(256), 0, st, src, dst, N,
                       m);
  return hipGetLastError();
}

int64_t back3_num_workgroups(int N) {
  return (int64_t)((N + kVX - 1) / kVX) * ((N + kVY - 1) / kVY) * ((N + kVZ - 1) / kVZ);
}

hipError_t launch_back3(const Back3Args& a, hipStream_t st) {
  const dim3 grid((a.N + kVX - 1) / kVX, (a.N + kVY - 1) / kVY, (a.N + kVZ - 1) / kVZ);
  if (a.v64)
    hipLaunchKernelGGL(back3_kernel<double>, grid, dim3(256), 0, st, a.geom, a.ids, a.N, a.n, a.v64,
                       a.out, a.lay[0], a.lay[1], a.lay[2], a.x, a.x_true, a.partials, a.mode,
                       a.ctl);
  else
    hipLaunchKernelGGL(back3_kernel<float>, grid, dim3(256), 0, st, a.geom, a.ids, a.N, a.n, a.v32,
                       a.out, a.lay[0], a.lay[1], a.lay[2], a.x, a.x_true, a.partials, a.mode,
                       a.ctl);
  return hipGetLastError();
}

int cg3_num_parts(int p) { return (p + 255) / 256; }

hipError_t launch_diag3(const DirGeom* geom, const DirList& ids, int N, int n, double lam,
                        double* minv, hipStream_t st) {
  if (ids.n <= 0) return hipSuccess;
  const int g = (n + kRT - 1) / kRT;
  hipLaunchKernelGGL(diag3_kernel, dim3(g, g, ids.n), dim3(256), 0, st, geom, ids, N, n, lam, minv);
  return hipGetLastError();
}

hipError_t launch_cg3_init(const double* e, const double* minv, double* r, double* pd, double* z,
                           int p, double* parts, int nparts_cap, double* sc, int* ctl, double tol2,
                           hipStream_t st) {
  const int np = cg3_num_parts(p);
  if (2 * np > nparts_cap) return hipErrorInvalidValue;
  hipLaunchKernelGGL(cg3_init_kernel, dim3(np), dim3(256), 0, st, e, minv, r, pd, z, p, parts);
  hipLaunchKernelGGL(cg3_start_kernel, dim3(1), dim3(256), 0, st, parts, np, sc, ctl, tol2);
  return hipGetLastError();
}

hipError_t launch_cg3_alpha(const double* dots, int nd, double* sc, int* ctl, hipStream_t st) {
  hipLaunchKernelGGL(cg3_alpha_kernel, dim3(1), dim3(256), 0, st, dots, nd, sc, ctl);
  return hipGetLastError();
}

hipError_t launch_cg3_update(double* z, double* r, const double* pd, const double* q,
                             const double* minv, int p, double* parts, double* sc, int* ctl,
                             hipStream_t st) {
  hipLaunchKernelGGL(cg3_update_kernel, dim3(cg3_num_parts(p)), dim3(256), 0, st, z, r, pd, q, minv,
                     p, parts, sc, ctl);
  return hipGetLastError();
}

hipError_t launch_cg3_beta(double* r, const double* minv, double* pd, int p, const double* parts,
                           double* sc, int* ctl, hipStream_t st) {
  hipLaunchKernelGGL(cg3_rr_kernel, dim3(1), dim3(256), 0, st, parts, cg3_num_parts(p), sc, ctl);
  hipLaunchKernelGGL(cg3_pd_kernel, dim3(cg3_num_parts(p)), dim3(256), 0, st, r, minv, pd, p, sc,
                     ctl);
  return hipGetLastError();
}

}  // namespace slim
