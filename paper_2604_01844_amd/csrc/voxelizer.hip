// Voxelizer (Eq. 2, Sec. 3.3) for gfx950: the density field sampled at the
// voxel centres of a regular grid, each Gaussian limited to its kappa-sigma
// ellipsoid, and its backward.
//
// Same structure as the rasterizer, one dimension up:
//   record kernel   per Gaussian: centre in voxel-index coordinates and rho
//                   (float4, the position+radius packing of Sec. 3.5), the
//                   voxel-unit inverse covariance pre-scaled by -log2(e)/2,
//                   half-extents in voxels and the 3D rectangle of 8^3-voxel
//                   tiles its box touches;
//   count kernel    one wave per Gaussian: of the rectangle's tiles, those
//                   its support ellipsoid actually reaches (exact box test;
//                   about 57% of the box's tiles for the standard scan);
//   scan / emit     keys of the reached tiles; the sort's value is the
//                   emission slot, whose Gaussian is gid[slot];
//   stable radix sort / ranges as in the rasterizer;
//   forward         one wave per 8^3 tile; each lane owns one x-row of 8
//                   voxels; records staged in LDS in batches of 64;
//   backward        one wave per tile; each lane owns one (tile, Gaussian)
//                   pair and sums the ten moments sum g e {1, d, d d^T} over
//                   the tile's 512 voxels into the pair's emission slot; per
//                   Gaussian, its contiguous slots are reduced in a fixed
//                   order and the chain rule applied.
#include "fgs_internal.h"

namespace fgs {
namespace {

constexpr int kVT = 8;     // voxel tile side
constexpr int kWave = 64;

struct __align__(16) Rect3 {
  unsigned short v[8];     // x0, y0, z0, x1, y1, z1, 0, 0
};

struct GridDev {
  float origin[3];
  const float *origin_dev;  // device copy of the origin read instead of origin[] (null: off)
  float h[3];
  int dims[3];
  int nt[3];               // tiles per axis
  float kappa;
  float tau;               // density-aware support threshold (0 = off)
};

// Voxel-unit quantities of one Gaussian: W = diag(h) R diag(1/s) is such
// that A_vox = W W^T is the inverse covariance in voxel-index units.
struct VoxGauss {
  float pv[3];             // centre in voxel-index coordinates
  float W[3][3];
  float A[3][3];
  float r[3];              // kap-sigma half-extents in voxels
};

__device__ __forceinline__ void vox_gauss(const GaussParams &P, const GridDev &G, float kap, VoxGauss &V) {
  for (int a = 0; a < 3; ++a) {
    const float o = G.origin_dev ? G.origin_dev[a] : G.origin[a];
    V.pv[a] = (P.p[a] - o) / G.h[a] - 0.5f;
    float var = 0.f;
    for (int j = 0; j < 3; ++j) {
      V.W[a][j] = G.h[a] * P.R[3 * a + j] / P.s[j];
      const float rs = P.R[3 * a + j] * P.s[j];
      var += rs * rs;
    }
    V.r[a] = kap * sqrtf(var) / G.h[a];
  }
  for (int a = 0; a < 3; ++a)
    for (int b = 0; b < 3; ++b)
      V.A[a][b] = V.W[a][0] * V.W[b][0] + V.W[a][1] * V.W[b][1] + V.W[a][2] * V.W[b][2];
}

__device__ __forceinline__ void vox_span(float c, float r, int n_tiles, int &t0, int &t1) {
#pragma clang fp contract(off)
  const float lim = 16777216.f;
  float lo = fminf(fmaxf(c - r, -lim), lim);
  float hi = fminf(fmaxf(c + r, -lim), lim);
  t0 = max(static_cast<int>(floorf(lo)) >> 3, 0);
  t1 = min(static_cast<int>(floorf(hi)) >> 3, n_tiles - 1);
}

// The tile culling test keeps tiles whose best voxel centre has
// d^2 <= k2 + kappa^2 (kCullSlack - 1), k2 the Gaussian's support bound (a
// Mahalanobis radius about 0.05% beyond the kappa support): a superset of the
// per-voxel test. On the pre-scaled exponent: arg >= thr_g + thr_widen, with
// thr_g the Gaussian's threshold (a1.z) and thr_widen = thr (kCullSlack - 1).
constexpr float kCullSlack = 1.001f;
constexpr float kLn2 = 0.6931471805599453f;

__global__ void zero_u64_kernel(unsigned long long *p, int n) {
  if (int(threadIdx.x) < n) p[threadIdx.x] = 0ull;
}

__global__ __launch_bounds__(256) void vox_record_kernel(fgs_gaussians g, GridDev G,
                                                         float4 *__restrict__ prho,
                                                         float4 *__restrict__ a0,
                                                         float4 *__restrict__ a1,
                                                         float4 *__restrict__ radii,
                                                         Rect3 *__restrict__ rect) {
  const int64_t i = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (i < g.n) {
    GaussParams P;
    load_gauss(g, i, P);
    // support on the pre-scaled exponent arg = -log2(e)/2 d^2: arg >= thr_g,
    // thr_g = -log2(e)/2 kappa^2, raised to log2(tau / rho) by the
    // density-aware support (d^2 <= min(kappa^2, 2 ln(rho / tau)), Sec. 3.5
    // boxes that also take the density into account); a Gaussian with
    // rho <= tau is left out
    const float k = -0.5f * kLog2e;
    float kap = G.kappa, thr_g = k * G.kappa * G.kappa;
    bool dropped = false;
    if (G.tau > 0.f) {
      if (P.rho > G.tau) {
        const float l2 = log2f(P.rho) - log2f(G.tau);
        thr_g = fmaxf(thr_g, -l2);
        const float k2t = 2.f * kLn2 * l2;
        if (k2t < kap * kap) kap = sqrtf(k2t);
      } else {
        dropped = true;
      }
    }
    VoxGauss V;
    vox_gauss(P, G, kap, V);
    prho[i] = make_float4(V.pv[0], V.pv[1], V.pv[2], P.rho);
    a0[i] = make_float4(k * V.A[0][0], 2.f * k * V.A[0][1], 2.f * k * V.A[0][2], k * V.A[1][1]);
    a1[i] = make_float4(2.f * k * V.A[1][2], k * V.A[2][2], thr_g, 0.f);
    radii[i] = make_float4(V.r[0], V.r[1], V.r[2], 0.f);
    int t0[3], t1[3];
    bool empty = dropped;
    for (int a = 0; a < 3; ++a) {
      vox_span(V.pv[a], V.r[a], G.nt[a], t0[a], t1[a]);
      empty |= t0[a] > t1[a];
    }
    Rect3 rc;
    if (empty || !isfinite(V.pv[0] + V.pv[1] + V.pv[2])) {
      for (int a = 0; a < 8; ++a) rc.v[a] = 0;
      rc.v[0] = rc.v[1] = rc.v[2] = 1;
    } else {
      for (int a = 0; a < 3; ++a) {
        rc.v[a] = static_cast<unsigned short>(t0[a]);
        rc.v[3 + a] = static_cast<unsigned short>(t1[a]);
      }
      rc.v[6] = rc.v[7] = 0;
    }
    rect[i] = rc;
  }
}

// Largest value of the pre-scaled (negative definite) form
// arg(d) = c0.x dx^2 + dx (c0.y dy + c0.z dz) + c0.w dy^2 + c1.x dy dz + c1.y dz^2
// over the box lo <= p + d <= hi. Its maximiser lies on one of the three
// planes x_a = clamp(p_a); on each, the restricted 2D form is maximised over
// the face rectangle along its two clamped lines (the same construction as
// the rasterizer's quadrant test, one dimension up).
__device__ float box_qmax(const float4 &c0, const float4 &c1, const float p[3], const float lo[3],
                          const float hi[3]) {
  const float M[3][3] = {{c0.x, 0.5f * c0.y, 0.5f * c0.z},
                         {0.5f * c0.y, c0.w, 0.5f * c1.x},
                         {0.5f * c0.z, 0.5f * c1.x, c1.y}};
  float best = -INFINITY;
#pragma unroll
  for (int a = 0; a < 3; ++a) {
    const int b = (a + 1) % 3, c = (a + 2) % 3;
    const float D = fminf(fmaxf(p[a], lo[a]), hi[a]) - p[a];
    const float lb = lo[b] - p[b], hb = hi[b] - p[b], lc = lo[c] - p[c], hc = hi[c] - p[c];
    const float mbb = M[b][b], mcc = M[c][c], mbc = M[b][c], mab = M[a][b], mac = M[a][c];
    const float det = mbb * mcc - mbc * mbc;
    if (!(det > 0.f)) return 0.f;  // degenerate form: keep the tile
    const float ybh = -D * (mcc * mab - mbc * mac) / det;
    const float ych = -D * (mbb * mac - mbc * mab) / det;
    const float yb1 = fminf(fmaxf(ybh, lb), hb);
    const float yc1 = fminf(fmaxf(-(mbc * yb1 + D * mac) / mcc, lc), hc);
    const float yc2 = fminf(fmaxf(ych, lc), hc);
    const float yb2 = fminf(fmaxf(-(mbc * yc2 + D * mab) / mbb, lb), hb);
    const float base = M[a][a] * D * D;
    const float f1 = base + 2.f * D * (mab * yb1 + mac * yc1) + yb1 * (mbb * yb1 + 2.f * mbc * yc1) + mcc * yc1 * yc1;
    const float f2 = base + 2.f * D * (mab * yb2 + mac * yc2) + yb2 * (mbb * yb2 + 2.f * mbc * yc2) + mcc * yc2 * yc2;
    best = fmaxf(best, fmaxf(f1, f2));
  }
  return best;
}

// Tile j (row-major, x fastest) of rectangle rc, and whether the Gaussian's
// support ellipsoid reaches one of its voxel centres (a superset test: the
// threshold carries a small slack).
// Tile j of the rectangle, row-major (x fastest).
__device__ __forceinline__ void tile_coords(const Rect3 &rc, uint32_t j, uint32_t &tx, uint32_t &ty, uint32_t &tz) {
  const uint32_t nx = uint32_t(rc.v[3]) - rc.v[0] + 1u, ny = uint32_t(rc.v[4]) - rc.v[1] + 1u;
  const uint32_t jz = j / (nx * ny);
  const uint32_t jxy = j - jz * nx * ny;
  const uint32_t jy = jxy / nx;
  tx = rc.v[0] + (jxy - jy * nx);
  ty = rc.v[1] + jy;
  tz = rc.v[2] + jz;
}

__device__ __forceinline__ bool tile_hit(const Rect3 &rc, uint32_t j, const float4 &p, const float4 &c0,
                                         const float4 &c1, float thr_cull, uint32_t &tx, uint32_t &ty,
                                         uint32_t &tz) {
  tile_coords(rc, j, tx, ty, tz);
  const float pc[3] = {p.x, p.y, p.z};
  const float lo[3] = {float(tx * kVT), float(ty * kVT), float(tz * kVT)};
  const float hi[3] = {lo[0] + float(kVT - 1), lo[1] + float(kVT - 1), lo[2] + float(kVT - 1)};
  return box_qmax(c0, c1, pc, lo, hi) >= thr_cull;
}

__device__ __forceinline__ uint32_t rect_tiles(const Rect3 &rc) {
  if (rc.v[0] > rc.v[3] || rc.v[1] > rc.v[4] || rc.v[2] > rc.v[5]) return 0u;
  return (uint32_t(rc.v[3]) - rc.v[0] + 1u) * (uint32_t(rc.v[4]) - rc.v[1] + 1u) * (uint32_t(rc.v[5]) - rc.v[2] + 1u);
}

// One wave per Gaussian: the number of tiles of its rectangle that its
// support reaches (the key count), and the 64-bit total. The hit ballots of
// the first kHitWords rounds are kept, so the emission reads them instead of
// repeating the test (rectangles of at most 64 kHitWords tiles).
constexpr int kHitWords = 8;

__global__ __launch_bounds__(256) void vox_count_kernel(int64_t n, const float4 *__restrict__ prho,
                                                        const float4 *__restrict__ a0,
                                                        const float4 *__restrict__ a1,
                                                        const Rect3 *__restrict__ rect, float thr_widen,
                                                        uint32_t *__restrict__ count,
                                                        unsigned long long *__restrict__ hits) {
  const int64_t i = int64_t(blockIdx.x) * 4 + (threadIdx.x >> 6);
  const int lane = threadIdx.x & 63;
  if (i >= n) return;
  const Rect3 rc = rect[i];
  const uint32_t nt = rect_tiles(rc);
  const float4 p = prho[i], c0 = a0[i], c1 = a1[i];
  const float thr_cull = c1.z + thr_widen;
  uint32_t cnt = 0;
  for (uint32_t j0 = 0; j0 < nt; j0 += 64) {
    const uint32_t j = j0 + lane;
    uint32_t tx, ty, tz;
    const bool hit = j < nt && tile_hit(rc, j, p, c0, c1, thr_cull, tx, ty, tz);
    const uint64_t bal = __ballot(hit);
    cnt += __popcll(bal);
    if (lane == 0 && nt <= 64u * kHitWords) hits[uint64_t(i) * kHitWords + j0 / 64] = bal;
  }
  if (lane == 0) count[i] = cnt;
}

// One wave per Gaussian: the keys of the tiles its support reaches, in
// row-major order, at its offset. The sort's value is the emission slot q
// (a Gaussian's slots are contiguous, which is where the backward writes its
// partial sums); gid[q] is the Gaussian.
__global__ __launch_bounds__(256) void vox_emit_kernel(int64_t n, int ntx, int nty, const float4 *__restrict__ prho,
                                                       const float4 *__restrict__ a0,
                                                       const float4 *__restrict__ a1,
                                                       const Rect3 *__restrict__ rect, float thr_widen,
                                                       const uint32_t *__restrict__ offset,
                                                       const unsigned long long *__restrict__ hits,
                                                       uint32_t *__restrict__ keys, uint32_t *__restrict__ vals,
                                                       uint32_t *__restrict__ gid, const uint32_t *__restrict__ kdev) {
  // nothing to emit: no pairs, or more than the lists were laid out for
  if (kdev[0] == 0u) return;
  const int64_t i = int64_t(blockIdx.x) * 4 + (threadIdx.x >> 6);
  const int lane = threadIdx.x & 63;
  if (i >= n) return;
  uint32_t o = offset[i];
  if (o == offset[i + 1]) return;
  const Rect3 rc = rect[i];
  const uint32_t nt = rect_tiles(rc);
  const float4 p = prho[i], c0 = a0[i], c1 = a1[i];
  const float thr_cull = c1.z + thr_widen;
  const uint64_t lt = (lane == 0) ? 0ull : (~0ull >> (64 - lane));
  const bool stored = nt <= 64u * kHitWords;  // the count kept this rectangle's ballots
  for (uint32_t j0 = 0; j0 < nt; j0 += 64) {
    const uint32_t j = j0 + lane;
    uint32_t tx = 0, ty = 0, tz = 0;
    bool hit;
    if (stored) {
      hit = j < nt && ((hits[uint64_t(i) * kHitWords + j0 / 64] >> lane) & 1ull);
      if (hit) tile_coords(rc, j, tx, ty, tz);
    } else {
      hit = j < nt && tile_hit(rc, j, p, c0, c1, thr_cull, tx, ty, tz);
    }
    const uint64_t bal = __ballot(hit);
    if (hit) {
      const uint32_t q = o + uint32_t(__popcll(bal & lt));
      keys[q] = (tz * uint32_t(nty) + ty) * uint32_t(ntx) + tx;
      vals[q] = q;
      gid[q] = uint32_t(i);
    }
    o += uint32_t(__popcll(bal));
  }
}

__global__ __launch_bounds__(256) void vox_ranges_kernel(const uint32_t *__restrict__ skeys, uint64_t K_cap,
                                                         const uint32_t *__restrict__ kdev, uint32_t T,
                                                         uint32_t *__restrict__ start) {
  const uint64_t K = min(K_cap, uint64_t(kdev[0]));
  const uint64_t k = uint64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (k > K) return;
  const int64_t prev = (k == 0) ? -1 : int64_t(skeys[k - 1]);
  const int64_t cur = (k == K) ? int64_t(T) : int64_t(skeys[k]);
  for (int64_t t = prev + 1; t <= cur; ++t) start[t] = uint32_t(k);
}

// kCount = true: count the (voxel, Gaussian) pairs in the support whose voxel
// lies in the grid (the algorithmic work) instead of writing the volume.
template <bool kCount, int TPB>
__global__ __launch_bounds__(kWave * TPB) void vox_fwd_kernel(const uint32_t *__restrict__ start,
                                                         const uint32_t *__restrict__ svals,
                                                         const float4 *__restrict__ prho,
                                                         const float4 *__restrict__ a0,
                                                         const float4 *__restrict__ a1,
                                                         const uint32_t *__restrict__ gid, GridDev G,
                                                         uint32_t n_tiles, int n_chunks,
                                                         float *__restrict__ vol,
                                                         unsigned long long *__restrict__ counter) {
  __shared__ float4 s_all[TPB][3][kWave];
  const int wid = threadIdx.x / kWave;
  float4 *s_p = s_all[wid][0], *s_a0 = s_all[wid][1], *s_a1 = s_all[wid][2];
  // work unit = (tile, chunk): chunk c takes batches c, c + n_chunks, ... of
  // the tile's list and writes its own partial volume (n_chunks > 1)
  const uint32_t unit = xcd_block(blockIdx.x, gridDim.x) * TPB + wid;
  if (unit >= n_tiles * uint32_t(n_chunks)) return;
  const uint32_t tile = unit / uint32_t(n_chunks);
  const uint32_t chunk = unit - tile * uint32_t(n_chunks);
  const int tx = int(tile % uint32_t(G.nt[0]));
  const int tyz = int(tile / uint32_t(G.nt[0]));
  const int ty = tyz % G.nt[1];
  const int tz = tyz / G.nt[1];
  const int lane = threadIdx.x & (kWave - 1);
  const int y = ty * kVT + (lane & 7);
  const int z = tz * kVT + (lane >> 3);
  const float fx0 = float(tx * kVT), fy = float(y), fz = float(z);
  float acc[kVT];
#pragma unroll
  for (int k = 0; k < kVT; ++k) acc[k] = 0.f;
  const uint32_t b0 = start[tile], e = start[tile + 1];
  for (uint32_t b = b0 + chunk * kWave; b < e; b += kWave * uint32_t(n_chunks)) {
    const uint32_t m = min(uint32_t(kWave), e - b);
    if (uint32_t(lane) < m) {
      const uint32_t r = gid[svals[b + lane]];
      s_p[lane] = prho[r];
      s_a0[lane] = a0[r];
      s_a1[lane] = a1[r];
    }
    wave_lds_sync();
    for (uint32_t j = 0; j < m; ++j) {
      const float4 p = s_p[j];
      const float4 c0 = s_a0[j];
      const float4 c1 = s_a1[j];
      const float dy = fy - p.y, dz = fz - p.z;
      const float B = fmaf(c0.y, dy, c0.z * dz);
      const float Cc = fmaf(dy, fmaf(c0.w, dy, c1.x * dz), c1.y * dz * dz);
      const float dx0 = fx0 - p.x;
      // exponent along the row, expanded about the first voxel:
      // arg(dx0 + k) = arg0 + k (2 a dx0 + B) + a k^2
      const float arg0 = fmaf(dx0, fmaf(c0.x, dx0, B), Cc);
      const float E = fmaf(2.f * c0.x, dx0, B);
#pragma unroll
      for (int k = 0; k < kVT; ++k) {
        const float fk = float(k);
        const float arg = (k == 0) ? arg0 : fmaf(fk, fmaf(c0.x, fk, E), arg0);
        if (kCount) {
          acc[k] += (arg >= c1.z) ? 1.f : 0.f;
        } else {
          const float ex = __builtin_amdgcn_exp2f(arg);
          acc[k] = fmaf(p.w, (arg >= c1.z) ? ex : 0.f, acc[k]);
        }
      }
    }
    wave_lds_sync();
  }
  if (kCount) {
    unsigned long long n = 0;
    if (y < G.dims[1] && z < G.dims[2]) {
#pragma unroll
      for (int k = 0; k < kVT; ++k)
        if (tx * kVT + k < G.dims[0]) n += static_cast<unsigned long long>(acc[k]);
    }
    for (int d = 32; d > 0; d >>= 1) n += __shfl_xor(n, d, 64);
    if (lane == 0 && n) atomicAdd(counter, n);
    return;
  }
  if (y < G.dims[1] && z < G.dims[2]) {
    const uint64_t n_vox = uint64_t(G.dims[0]) * uint64_t(G.dims[1]) * uint64_t(G.dims[2]);
    float *row = vol + uint64_t(chunk) * n_vox + (uint64_t(z) * G.dims[1] + y) * uint64_t(G.dims[0]);
#pragma unroll
    for (int k = 0; k < kVT; ++k) {
      const int x = tx * kVT + k;
      if (x < G.dims[0]) row[x] = acc[k];
    }
  }
}

// Backward over one 8^3 tile: lane j owns pair (tile, list[j]) and sums the
// ten moments over the 512 voxels. Coordinates are relative to the tile
// centre, (cx, cy, cz) in {-3.5, ..., 3.5}; along each x-row the exponent is
// a quadratic in cx with lane coefficients. The tile's g and g cx are staged
// in LDS, and each voxel adds g e into its column's sum (over y and z) and
// into the row's sums of g e and g e cx (three FMAs); the x-moments follow
// from the column sums, the others from the row sums, and all are moved to
// the Gaussian's centre once per pair. Branch-free loop body.
template <int TPB>
__global__ __launch_bounds__(kWave * TPB) void vox_bwd_kernel(const uint32_t *__restrict__ start,
                                                         const uint32_t *__restrict__ svals,
                                                         const float4 *__restrict__ prho,
                                                         const float4 *__restrict__ a0,
                                                         const float4 *__restrict__ a1,
                                                         const uint32_t *__restrict__ gid,
                                                         GridDev G, uint32_t n_tiles, int n_chunks,
                                                         const float *__restrict__ gvol,
                                                         float2 *__restrict__ partials) {
  __shared__ float4 s_g4_all[TPB][2][kVT * kVT * kVT / 4];
  const int wid = threadIdx.x / kWave;
  float4 *s_g4 = s_g4_all[wid][0];
  float *s_g = reinterpret_cast<float *>(s_g4);
  const float h = 0.5f * (kVT - 1);
  // work unit = (tile, chunk): chunk c takes batches c, c + n_chunks, ...
  // (the natural block order: the XCD-aware one measured 4% slower here)
  const uint32_t unit = blockIdx.x * TPB + wid;
  if (unit >= n_tiles * uint32_t(n_chunks)) return;
  const uint32_t tile = unit / uint32_t(n_chunks);
  const uint32_t chunk = unit - tile * uint32_t(n_chunks);
  const int tx = int(tile % uint32_t(G.nt[0]));
  const int tyz = int(tile / uint32_t(G.nt[0]));
  const int ty = tyz % G.nt[1];
  const int tz = tyz / G.nt[1];
  const int lane = threadIdx.x & (kWave - 1);
  for (int q = lane; q < kVT * kVT * kVT; q += kWave) {
    const int x = tx * kVT + (q & 7), y = ty * kVT + ((q >> 3) & 7), z = tz * kVT + (q >> 6);
    const float g = (x < G.dims[0] && y < G.dims[1] && z < G.dims[2])
                        ? gvol[(uint64_t(z) * G.dims[1] + y) * uint64_t(G.dims[0]) + x]
                        : 0.f;
    s_g[q] = g;
    s_g[kVT * kVT * kVT + q] = g * (float(q & 7) - h);
  }
  wave_lds_sync();
  const uint32_t b0 = start[tile], e = start[tile + 1];
  const float ox = float(tx * kVT) + h, oy = float(ty * kVT) + h, oz = float(tz * kVT) + h;
  for (uint32_t b = b0 + chunk * kWave; b < e; b += kWave * uint32_t(n_chunks)) {
    const uint32_t k = b + lane;
    const bool active = k < e;
    float4 p = make_float4(ox, oy, oz, 0.f), c0 = make_float4(0.f, 0.f, 0.f, 0.f), c1 = c0;
    uint32_t q = 0;
    if (active) {
      q = svals[k];
      const uint32_t r = gid[q];
      p = prho[r];
      c0 = a0[r];
      c1 = a1[r];
    }
    const float qx = p.x - ox, qy = p.y - oy, qz = p.z - oz;
    const float m2aqx = -2.f * c0.x * qx;
    const float aqx2 = c0.x * qx * qx;
    float A[kVT];
#pragma unroll
    for (int u = 0; u < kVT; ++u) A[u] = 0.f;
    float Sy = 0.f, Sz = 0.f, Sxy = 0.f, Sxz = 0.f, Syy = 0.f, Syz = 0.f, Szz = 0.f;
    for (int zz = 0; zz < kVT; ++zz) {
      const float cz = float(zz) - h;
      const float dz = cz - qz;
#pragma unroll 2
      for (int yy = 0; yy < kVT; ++yy) {
        const float cy = float(yy) - h;
        const float dy = cy - qy;
        const float lin = fmaf(c0.y, dy, c0.z * dz);
        const float Cc = fmaf(dy, fmaf(c0.w, dy, c1.x * dz), c1.y * dz * dz);
        const float brow = lin + m2aqx;
        const float drow = fmaf(-lin, qx, aqx2 + Cc);
        const float4 *g4 = s_g4 + (zz * kVT + yy) * (kVT / 4);
        float R0 = 0.f, R1 = 0.f;
#pragma unroll
        for (int qd = 0; qd < kVT / 4; ++qd) {
          const float4 g0 = g4[qd];
          const float4 g1 = g4[kVT * kVT * kVT / 4 + qd];
          const float G0[4] = {g0.x, g0.y, g0.z, g0.w};
          const float G1[4] = {g1.x, g1.y, g1.z, g1.w};
#pragma unroll
          for (int u = 0; u < 4; ++u) {
            const float cx = float(qd * 4 + u) - h;
            const float arg = fmaf(cx, fmaf(c0.x, cx, brow), drow);
            const float ex = (arg >= c1.z) ? __builtin_amdgcn_exp2f(arg) : 0.f;
            A[qd * 4 + u] = fmaf(G0[u], ex, A[qd * 4 + u]);
            R0 = fmaf(G0[u], ex, R0);
            R1 = fmaf(G1[u], ex, R1);
          }
        }
        Sy = fmaf(R0, cy, Sy);
        Sz = fmaf(R0, cz, Sz);
        Sxy = fmaf(R1, cy, Sxy);
        Sxz = fmaf(R1, cz, Sxz);
        const float R0y = R0 * cy;
        Syy = fmaf(R0y, cy, Syy);
        Syz = fmaf(R0y, cz, Syz);
        Szz = fmaf(R0 * cz, cz, Szz);
      }
    }
    float S0 = 0.f, Sc = 0.f, Scc = 0.f;
#pragma unroll
    for (int u = 0; u < kVT; ++u) {
      const float cx = float(u) - h;
      S0 += A[u];
      Sc = fmaf(A[u], cx, Sc);
      Scc = fmaf(A[u], cx * cx, Scc);
    }
    if (active) {
      // moments about the Gaussian centre: d = c - q
      const float Mx = fmaf(-qx, S0, Sc);
      const float My = fmaf(-qy, S0, Sy);
      const float Mz = fmaf(-qz, S0, Sz);
      const float Mxx = fmaf(qx * qx, S0, fmaf(-2.f * qx, Sc, Scc));
      const float Myy = fmaf(qy * qy, S0, fmaf(-2.f * qy, Sy, Syy));
      const float Mzz = fmaf(qz * qz, S0, fmaf(-2.f * qz, Sz, Szz));
      const float Mxy = fmaf(qx * qy, S0, fmaf(-qy, Sc, fmaf(-qx, Sy, Sxy)));
      const float Mxz = fmaf(qx * qz, S0, fmaf(-qz, Sc, fmaf(-qx, Sz, Sxz)));
      const float Myz = fmaf(qy * qz, S0, fmaf(-qz, Sy, fmaf(-qy, Sz, Syz)));
      partials[5 * uint64_t(q) + 0] = make_float2(S0, Mx);
      partials[5 * uint64_t(q) + 1] = make_float2(My, Mz);
      partials[5 * uint64_t(q) + 2] = make_float2(Mxx, Mxy);
      partials[5 * uint64_t(q) + 3] = make_float2(Mxz, Myy);
      partials[5 * uint64_t(q) + 4] = make_float2(Myz, Mzz);
    }
  }
}

// Per Gaussian: reduce its contiguous partial slots (ten moments each), then
// the chain rule. A block takes kGradGauss consecutive Gaussians; their slots
// are read by groups of kGradLanes lanes (consecutive lanes, consecutive
// slots) and summed across the group in a fixed butterfly order; one thread
// per Gaussian then applies the chain rule.
constexpr int kGradGauss = 64;
constexpr int kGradLanes = 32;

__global__ __launch_bounds__(256) void vox_grad_kernel(fgs_gaussians g, GridDev G,
                                                       const uint32_t *__restrict__ offset,
                                                       const float2 *__restrict__ partials,
                                                       const uint32_t *__restrict__ kdev,
                                                       fgs_gaussian_grads out, int accumulate) {
  __shared__ float s_sum[kGradGauss][11];
  __shared__ uint32_t s_off[kGradGauss + 1];
  // kdev[1]: the lists overflowed their capacity and hold nothing
  const bool none = kdev[1] != 0u;
  const int t = threadIdx.x;
  const int64_t i0 = int64_t(blockIdx.x) * kGradGauss;
  // the block's offsets in one coalesced read (offset has n + 1 entries)
  if (t <= kGradGauss && i0 + t <= g.n) s_off[t] = offset[i0 + t];
  __syncthreads();
  const int li = t % kGradLanes;
  for (int idx = t / kGradLanes; idx < kGradGauss; idx += 256 / kGradLanes) {
    if (i0 + idx >= g.n || none) break;
    const uint32_t o = s_off[idx], end = s_off[idx + 1];
    if (o == end) continue;  // the whole lane group agrees: no pairs, nothing to sum
    float acc[10];
#pragma unroll
    for (int c = 0; c < 10; ++c) acc[c] = 0.f;
    {
      for (uint32_t q = o + li; q < end; q += kGradLanes) {
#pragma unroll
        for (int c = 0; c < 5; ++c) {
          const float2 v = partials[5 * uint64_t(q) + c];
          acc[2 * c] += v.x;
          acc[2 * c + 1] += v.y;
        }
      }
    }
#pragma unroll
    for (int d = 1; d < kGradLanes; d <<= 1)
#pragma unroll
      for (int c = 0; c < 10; ++c) acc[c] += __shfl_xor(acc[c], d, kGradLanes);
    if (li == 0)
#pragma unroll
      for (int c = 0; c < 10; ++c) s_sum[idx][c] = acc[c];
  }
  __syncthreads();
  if (t >= kGradGauss) return;
  const int64_t i = i0 + t;
  if (i >= g.n) return;
  const int64_t n = g.n;
  const uint32_t o = s_off[t], end = none ? o : s_off[t + 1];
  // a Gaussian with no pair adds nothing: when accumulating, leave it alone
  if (accumulate && o == end) return;
  float s[10];
#pragma unroll
  for (int c = 0; c < 10; ++c) s[c] = s_sum[t][c];
  float res[11];
#pragma unroll
  for (int c = 0; c < 11; ++c) res[c] = 0.f;
  if (o != end) {
    GaussParams P;
    load_gauss(g, i, P);
    VoxGauss V;
    vox_gauss(P, G, G.kappa, V);
    // s: S0, Sx, Sy, Sz, Sxx, Sxy, Sxz, Syy, Syz, Szz with d = voxel - centre
    const float rho = P.rho;
    const float Sd[3] = {s[1], s[2], s[3]};
    for (int a = 0; a < 3; ++a) {
      const float dpv = rho * (V.A[a][0] * Sd[0] + V.A[a][1] * Sd[1] + V.A[a][2] * Sd[2]);
      res[a] = dpv / G.h[a];
    }
    // dA_vox = -rho/2 M, M the symmetric second-moment matrix
    const float M[3][3] = {{s[4], s[5], s[6]}, {s[5], s[7], s[8]}, {s[6], s[8], s[9]}};
    // A_vox = W W^T: dW = 2 dA W
    float dR[9];
    for (int j = 0; j < 3; ++j) {
      float dls = 0.f;
      for (int a = 0; a < 3; ++a) {
        const float dW = -rho * (M[a][0] * V.W[0][j] + M[a][1] * V.W[1][j] + M[a][2] * V.W[2][j]);
        // W[a][j] = h_a R[a][j] / s_j
        dR[3 * a + j] = dW * G.h[a] / P.s[j];
        dls -= dW * V.W[a][j];
      }
      res[3 + j] = dls;
    }
    float dq[4];
    rot_grad_to_quat(P.qh, P.qnorm, dR, dq);
    res[6] = dq[0]; res[7] = dq[1]; res[8] = dq[2]; res[9] = dq[3];
    res[10] = s[0];
  }
  if (accumulate) {
    res[0] += out.mean[i]; res[1] += out.mean[n + i]; res[2] += out.mean[2 * n + i];
    res[3] += out.log_scale[i]; res[4] += out.log_scale[n + i]; res[5] += out.log_scale[2 * n + i];
    res[6] += out.quat[i]; res[7] += out.quat[n + i]; res[8] += out.quat[2 * n + i]; res[9] += out.quat[3 * n + i];
    res[10] += out.density[i];
  }
  out.mean[i] = res[0]; out.mean[n + i] = res[1]; out.mean[2 * n + i] = res[2];
  out.log_scale[i] = res[3]; out.log_scale[n + i] = res[4]; out.log_scale[2 * n + i] = res[5];
  out.quat[i] = res[6]; out.quat[n + i] = res[7]; out.quat[2 * n + i] = res[8]; out.quat[3 * n + i] = res[9];
  out.density[i] = res[10];
}

// ------------------------------------------------------------------ host

struct VoxLayout {
  uint64_t N, T, K;
  uint64_t total64, kdev, prho, radii, rect, offset, a0, a1, scan_scratch, start, hits;
  uint64_t fixed_end;
  uint64_t keys, vals, keys_alt, vals_alt, gid, sort_scratch, partials;
  uint64_t total;
  bool sorted_in_alt;
};

VoxLayout vox_layout(uint64_t N, uint64_t T, uint64_t K) {
  VoxLayout L{};
  L.N = N;
  L.T = T;
  L.K = K;
  Carver c(nullptr);
  c.take<unsigned long long>(1, &L.total64);
  c.take<uint32_t>(4, &L.kdev);
  c.take<float4>(N, &L.prho);
  c.take<float4>(N, &L.radii);
  c.take<Rect3>(N, &L.rect);
  c.take<uint32_t>(N + 1, &L.offset);
  c.take<float4>(N, &L.a0);
  c.take<float4>(N, &L.a1);
  c.take<uint32_t>(scan_scratch_words(N), &L.scan_scratch);
  c.take<uint32_t>(T + 1, &L.start);
  c.take<unsigned long long>(N * kHitWords, &L.hits);
  L.fixed_end = c.used;
  c.take<uint32_t>(K, &L.keys);
  c.take<uint32_t>(K, &L.vals);
  c.take<uint32_t>(K, &L.keys_alt);
  c.take<uint32_t>(K, &L.vals_alt);
  c.take<uint32_t>(K, &L.gid);
  c.take<uint32_t>(sort_scratch_words(K), &L.sort_scratch);
  c.take<float>(10 * K, &L.partials);
  L.total = c.used;
  const int bits = bits_for(T);
  const int passes = sort_passes(K, bits);
  L.sorted_in_alt = (passes & 1) != 0;
  return L;
}

template <typename T>
T *at(void *base, uint64_t off) {
  return reinterpret_cast<T *>(static_cast<char *>(base) + off);
}

int validate(const fgs_gaussians *g, const fgs_grid *grid, const fgs_opts *o, fgs_workspace *ws) {
  if (!g || !grid || !o || !ws) return fail(FGS_E_INVALID, "null argument");
  if (g->n <= 0 || !g->mean || !g->log_scale || !g->quat || !g->density)
    return fail(FGS_E_INVALID, "invalid Gaussians");
  if (g->n > 0x7fffffff) return fail(FGS_E_UNSUPPORTED, "more than 2^31 Gaussians");
  for (int a = 0; a < 3; ++a) {
    if (grid->dims[a] <= 0 || grid->dims[a] > 65535 * kVT) return fail(FGS_E_INVALID, "grid dims");
    if (!(grid->spacing[a] > 0.f)) return fail(FGS_E_INVALID, "grid spacing");
  }
  if (!(o->kappa > 0.f)) return fail(FGS_E_INVALID, "kappa must be > 0");
  if (o->model != 0) return fail(FGS_E_INVALID, "opts.model must be 0 for the voxelizer");
  if (!(o->density_aabb_tau >= 0.f) || !std::isfinite(o->density_aabb_tau))
    return fail(FGS_E_INVALID, "density_aabb_tau must be finite and >= 0");
  return FGS_OK;
}

GridDev make_grid_dev(const fgs_grid *grid, const fgs_opts *o) {
  GridDev G{};
  for (int a = 0; a < 3; ++a) {
    G.origin[a] = grid->origin[a];
    G.h[a] = grid->spacing[a];
    G.dims[a] = grid->dims[a];
    G.nt[a] = (grid->dims[a] + kVT - 1) / kVT;
  }
  G.kappa = o->kappa;
  G.tau = o->density_aabb_tau;
  G.origin_dev = nullptr;
  return G;
}

// extra_bytes: room the caller needs after the lists (partial volumes).
int vox_build(const fgs_gaussians *g, const fgs_grid *grid, const fgs_opts *o, fgs_workspace *ws,
              hipStream_t s, VoxLayout *Lout, GridDev *Gout, uint64_t extra_bytes = 0,
              const float *origin_dev = nullptr) {
  GridDev G = make_grid_dev(grid, o);
  G.origin_dev = origin_dev;
  const uint64_t T = uint64_t(G.nt[0]) * G.nt[1] * G.nt[2];
  if (T >= 0xffffffffull) return fail(FGS_E_UNSUPPORTED, "too many voxel tiles");
  const uint64_t N = uint64_t(g->n);
  // key_capacity > 0: lists laid out for that many pairs, count kept on the device
  const uint64_t cap = ws->key_capacity;
  if (cap >= 0xffffffffull) return fail(FGS_E_UNSUPPORTED, "key_capacity must be below 2^32");
  VoxLayout L = vox_layout(N, T, cap);
  ws->kind = 0;
  if (cap > 0) {
    ws->needed = L.total + extra_bytes;
    ws->n_pairs = cap;
    ws->n_records = N;
    ws->n_tiles = T;
    if (!ws->ptr || ws->bytes < ws->needed) return fail(FGS_E_CAPACITY, "workspace too small for key_capacity pairs");
  } else if (!ws->ptr || ws->bytes < L.fixed_end + (uint64_t(1) << 20)) {
    ws->needed = L.fixed_end + (uint64_t(64) << 20);
    return fail(FGS_E_CAPACITY, "workspace too small for the per-Gaussian arrays");
  }
  void *b = ws->ptr;
  unsigned long long *total64 = at<unsigned long long>(b, L.total64);
  vox_record_kernel<<<grid_for(N, 256), 256, 0, s>>>(*g, G, at<float4>(b, L.prho), at<float4>(b, L.a0),
                                                      at<float4>(b, L.a1), at<float4>(b, L.radii),
                                                      at<Rect3>(b, L.rect));
  FGS_LAUNCH_CHECK("vox_record_kernel");
  const float thr_widen = -0.5f * kLog2e * o->kappa * o->kappa * (kCullSlack - 1.f);
  vox_count_kernel<<<grid_for(N, 4), 256, 0, s>>>(int64_t(N), at<float4>(b, L.prho), at<float4>(b, L.a0),
                                                   at<float4>(b, L.a1), at<Rect3>(b, L.rect), thr_widen,
                                                   at<uint32_t>(b, L.offset), at<unsigned long long>(b, L.hits));
  FGS_LAUNCH_CHECK("vox_count_kernel");
  // offsets, the 64-bit pair total and the device pair count (0 past the
  // capacity) in one scan
  uint32_t *kdev = at<uint32_t>(b, L.kdev);
  int st = scan_counts(at<uint32_t>(b, L.offset), N, at<uint32_t>(b, L.scan_scratch),
                       cap > 0 ? cap : uint64_t(0xfffffffeull), total64, kdev, cap > 0 ? ws->overflow : nullptr, s);
  if (st != FGS_OK) return st;
  if (cap == 0) {
    unsigned long long K64 = 0;
    FGS_HIP(hipMemcpyAsync(&K64, total64, sizeof(K64), hipMemcpyDeviceToHost, s));
    FGS_HIP(hipStreamSynchronize(s));
    if (K64 >= 0xffffffffull)
      return fail(FGS_E_UNSUPPORTED, "more than 2^32 (tile, Gaussian) pairs; split the grid into slabs");
    const uint64_t K = K64;
    L = vox_layout(N, T, K);
    ws->needed = L.total + extra_bytes;
    ws->n_pairs = K;
    ws->n_records = N;
    ws->n_tiles = T;
    if (ws->bytes < L.total + extra_bytes) return fail(FGS_E_CAPACITY, "workspace too small for the tile lists");
  }
  const uint64_t K = L.K;
  if (K > 0) {
    vox_emit_kernel<<<grid_for(N, 4), 256, 0, s>>>(int64_t(N), G.nt[0], G.nt[1], at<float4>(b, L.prho),
                                                    at<float4>(b, L.a0), at<float4>(b, L.a1), at<Rect3>(b, L.rect),
                                                    thr_widen, at<uint32_t>(b, L.offset),
                                                    at<unsigned long long>(b, L.hits), at<uint32_t>(b, L.keys),
                                                    at<uint32_t>(b, L.vals), at<uint32_t>(b, L.gid), kdev);
    FGS_LAUNCH_CHECK("vox_emit_kernel");
  }
  uint32_t *sk, *sv;
  st = radix_sort_pairs(at<uint32_t>(b, L.keys), at<uint32_t>(b, L.vals), at<uint32_t>(b, L.keys_alt),
                        at<uint32_t>(b, L.vals_alt), K, bits_for(T), at<uint32_t>(b, L.sort_scratch),
                        &sk, &sv, s, kSortMaxBits, cap > 0 ? kdev : nullptr);
  if (st != FGS_OK) return st;
  vox_ranges_kernel<<<grid_for(K + 1, 256), 256, 0, s>>>(sk, K, kdev, uint32_t(T), at<uint32_t>(b, L.start));
  FGS_LAUNCH_CHECK("vox_ranges_kernel");
  ws->kind = 2;
  *Lout = L;
  *Gout = G;
  return FGS_OK;
}

}  // namespace

// Workspace of a voxelizer call: as rast_workspace_bytes (the forward over
// few tiles also keeps one partial volume per chunk).
int vox_workspace_bytes(const fgs_gaussians *g, const fgs_grid *grid, bool forward, uint64_t *fixed_bytes,
                        uint64_t *bytes_per_key) {
  if (!g || !grid || g->n <= 0 || grid->dims[0] <= 0 || grid->dims[1] <= 0 || grid->dims[2] <= 0)
    return fail(FGS_E_INVALID, "workspace query: null argument, no Gaussians or grid dims");
  const uint64_t T = uint64_t((grid->dims[0] + kVT - 1) / kVT) * uint64_t((grid->dims[1] + kVT - 1) / kVT) *
                     uint64_t((grid->dims[2] + kVT - 1) / kVT);
  const uint64_t N = uint64_t(g->n);
  const uint64_t k_ref = uint64_t(1) << 24;
  const uint64_t base = vox_layout(N, T, 0).total;
  const uint64_t big = vox_layout(N, T, k_ref).total;
  const int chunks = chunks_per_tile(T);
  const uint64_t n_vox = uint64_t(grid->dims[0]) * uint64_t(grid->dims[1]) * uint64_t(grid->dims[2]);
  const uint64_t part = (forward && chunks > 1) ? uint64_t(chunks) * n_vox * sizeof(float) + 256 : 0;
  // (a call first asks for the per-record arrays plus 1 MiB before it knows K)
  *fixed_bytes = base + part + 8 * kAlign + (uint64_t(1) << 20);
  *bytes_per_key = (big - base + k_ref - 1) / k_ref;
  return FGS_OK;
}

int vox_binning_layout(const fgs_workspace *ws, uint64_t off[9], uint64_t counts[3]) {
  VoxLayout L = vox_layout(ws->n_records, ws->n_tiles, ws->n_pairs);
  off[0] = L.prho;
  off[1] = L.radii;
  off[2] = L.rect;
  off[3] = L.offset;
  off[4] = L.sorted_in_alt ? L.keys : L.keys_alt;
  off[5] = L.sorted_in_alt ? L.vals : L.vals_alt;
  off[6] = L.sorted_in_alt ? L.keys_alt : L.keys;
  off[7] = L.sorted_in_alt ? L.vals_alt : L.vals;
  off[8] = L.start;
  counts[0] = L.N;
  counts[1] = L.K;
  counts[2] = L.T;
  return FGS_OK;
}

}  // namespace fgs

namespace fgs {

int vox_forward(const fgs_gaussians *g, const fgs_grid *grid, const fgs_opts *opts, float *vol, fgs_workspace *ws,
                hipStream_t s, const float *origin_dev) {
  int st = validate(g, grid, opts, ws);
  if (st != FGS_OK) return st;
  if (!vol) return fail(FGS_E_INVALID, "null volume");
  const uint64_t n_tiles = uint64_t((grid->dims[0] + kVT - 1) / kVT) * uint64_t((grid->dims[1] + kVT - 1) / kVT) *
                           uint64_t((grid->dims[2] + kVT - 1) / kVT);
  const int chunks = chunks_per_tile(n_tiles);
  const uint64_t n_vox = uint64_t(grid->dims[0]) * uint64_t(grid->dims[1]) * uint64_t(grid->dims[2]);
  // partial volumes of the chunks, after the lists (only when chunked)
  const uint64_t part_bytes = chunks > 1 ? uint64_t(chunks) * n_vox * sizeof(float) + 256 : 0;
  VoxLayout L;
  GridDev G;
  st = vox_build(g, grid, opts, ws, s, &L, &G, part_bytes, origin_dev);
  if (st != FGS_OK) return st;
  void *b = ws->ptr;
  float *part = chunks > 1 ? at<float>(b, (L.total + 255) / 256 * 256) : vol;
  const uint32_t *sv = at<uint32_t>(b, L.sorted_in_alt ? L.vals_alt : L.vals);
  hipEvent_t *ev = static_cast<hipEvent_t *>(opts->events);
  if (ev) FGS_HIP(hipEventRecord(ev[0], s));
  const uint64_t units = L.T * uint64_t(chunks);
  with_tiles_per_block(units, [&](auto tpb) {
    constexpr int TPB = decltype(tpb)::value;
    vox_fwd_kernel<false, TPB><<<grid_for(units, TPB), kWave * TPB, 0, s>>>(
        at<uint32_t>(b, L.start), sv, at<float4>(b, L.prho), at<float4>(b, L.a0), at<float4>(b, L.a1),
        at<uint32_t>(b, L.gid), G, uint32_t(L.T), chunks, part, nullptr);
  });
  FGS_LAUNCH_CHECK("vox_fwd_kernel");
  if (chunks > 1) {
    st = sum_chunks(part, chunks, n_vox, vol, s);
    if (st != FGS_OK) return st;
  }
  if (ev) FGS_HIP(hipEventRecord(ev[1], s));
  return FGS_OK;
}

}  // namespace fgs

using namespace fgs;

extern "C" int fgs_voxelize_fwd(const fgs_gaussians *g, const fgs_grid *grid, const fgs_opts *opts,
                                float *vol, fgs_workspace *ws, void *stream) {
  return vox_forward(g, grid, opts, vol, ws, static_cast<hipStream_t>(stream), nullptr);
}

extern "C" int fgs_voxelize_support(const fgs_gaussians *g, const fgs_grid *grid, const fgs_opts *opts,
                                    uint64_t *out, fgs_workspace *ws, void *stream) {
  int st = validate(g, grid, opts, ws);
  if (st != FGS_OK) return st;
  if (!out) return fail(FGS_E_INVALID, "null output");
  hipStream_t s = static_cast<hipStream_t>(stream);
  VoxLayout L;
  GridDev G;
  st = vox_build(g, grid, opts, ws, s, &L, &G);
  if (st != FGS_OK) return st;
  void *b = ws->ptr;
  unsigned long long *cnt = reinterpret_cast<unsigned long long *>(out);
  zero_u64_kernel<<<1, 1, 0, s>>>(cnt, 1);
  FGS_LAUNCH_CHECK("zero_u64_kernel");
  const uint32_t *sv = at<uint32_t>(b, L.sorted_in_alt ? L.vals_alt : L.vals);
  const int chunks = chunks_per_tile(L.T);
  const uint64_t units = L.T * uint64_t(chunks);
  with_tiles_per_block(units, [&](auto tpb) {
    constexpr int TPB = decltype(tpb)::value;
    vox_fwd_kernel<true, TPB><<<grid_for(units, TPB), kWave * TPB, 0, s>>>(
        at<uint32_t>(b, L.start), sv, at<float4>(b, L.prho), at<float4>(b, L.a0), at<float4>(b, L.a1),
        at<uint32_t>(b, L.gid), G, uint32_t(L.T), chunks, nullptr, cnt);
  });
  FGS_LAUNCH_CHECK("vox_fwd_kernel<count>");
  return FGS_OK;
}

namespace fgs {

int vox_backward(const fgs_gaussians *g, const fgs_grid *grid, const fgs_opts *opts, const float *grad_vol,
                 fgs_gaussian_grads *out, fgs_workspace *ws, hipStream_t s, const float *origin_dev) {
  int st = validate(g, grid, opts, ws);
  if (st != FGS_OK) return st;
  if (!grad_vol || !out || !out->mean || !out->log_scale || !out->quat || !out->density)
    return fail(FGS_E_INVALID, "null gradient buffer");
  VoxLayout L;
  GridDev G;
  if (opts->recompute) {
    st = vox_build(g, grid, opts, ws, s, &L, &G, 0, origin_dev);
    if (st != FGS_OK) return st;
  } else {
    G = make_grid_dev(grid, opts);
    G.origin_dev = origin_dev;
    const uint64_t T = uint64_t(G.nt[0]) * G.nt[1] * G.nt[2];
    if (ws->kind != 2 || ws->n_records != uint64_t(g->n) || ws->n_tiles != T || !ws->ptr)
      return fail(FGS_E_INVALID, "workspace does not hold this call's voxelizer lists");
    L = vox_layout(uint64_t(g->n), T, ws->n_pairs);
    if (ws->bytes < L.total) return fail(FGS_E_INVALID, "workspace lists do not match this call");
  }
  void *b = ws->ptr;
  const uint32_t *sv = at<uint32_t>(b, L.sorted_in_alt ? L.vals_alt : L.vals);
  hipEvent_t *ev = static_cast<hipEvent_t *>(opts->events);
  if (ev) FGS_HIP(hipEventRecord(ev[0], s));
  if (L.K > 0) {
    const int chunks = chunks_per_tile(L.T);
    const uint64_t units = L.T * uint64_t(chunks);
    with_tiles_per_block(units, [&](auto tpb) {
      constexpr int TPB = decltype(tpb)::value;
      vox_bwd_kernel<TPB><<<grid_for(units, TPB), kWave * TPB, 0, s>>>(
          at<uint32_t>(b, L.start), sv, at<float4>(b, L.prho), at<float4>(b, L.a0), at<float4>(b, L.a1),
          at<uint32_t>(b, L.gid), G, uint32_t(L.T), chunks, grad_vol, at<float2>(b, L.partials));
    });
    FGS_LAUNCH_CHECK("vox_bwd_kernel");
  }
  if (ev) FGS_HIP(hipEventRecord(ev[1], s));
  vox_grad_kernel<<<grid_for(uint64_t(g->n), kGradGauss), 256, 0, s>>>(*g, G, at<uint32_t>(b, L.offset),
                                                                at<float2>(b, L.partials),
                                                                at<uint32_t>(b, L.kdev), *out,
                                                                opts->accumulate);
  FGS_LAUNCH_CHECK("vox_grad_kernel");
  return FGS_OK;
}

}  // namespace fgs

extern "C" int fgs_voxelize_bwd(const fgs_gaussians *g, const fgs_grid *grid, const fgs_opts *opts,
                                const float *grad_vol, fgs_gaussian_grads *out, fgs_workspace *ws,
                                void *stream) {
  return vox_backward(g, grid, opts, grad_vol, out, ws, static_cast<hipStream_t>(stream), nullptr);
}
