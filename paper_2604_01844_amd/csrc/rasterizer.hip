// X-ray rasterizer (Eq. 3-4, Sec. 3.2; accelerations of Sec. 3.5) for gfx950.
//
// Forward, per call over a batch of views:
//   1. record kernel      one thread per (view, Gaussian): splat centre,
//                         pre-scaled conic and w = rho mu (float4), support
//                         half-extents, axis-aligned tile rectangle, count.
//   2. exclusive scan     counts -> key offsets (one readback of the total).
//   3. emit kernel        keys (view * tiles_per_view + tile) and values
//                         (record index), row-major inside each rectangle.
//   4. radix sort         stable; no depth key (the sum is order-free).
//   5. ranges kernel      per-tile [start, end) by boundary detection.
//   6. splat kernel       one 64-lane wave per 16x16 tile; batches of 64
//                         records staged in LDS; each lane owns a column of
//                         4 pixels; the Gaussian factor is one v_exp_f32 of a
//                         pre-scaled quadratic form; support test d^2 <= k^2.
// Backward (per-Gaussian formulation, Sec. 3.5):
//   7. splat-grad kernel  one wave per tile; each lane owns one
//                         (tile, Gaussian) pair of the tile's list and sums
//                         over the 256 pixels, reading dL/dI from LDS, the
//                         six moments sum g e {1, dx, dy, dx^2, dx dy, dy^2}.
//                         No atomics and no cross-lane traffic: the pair's
//                         sums go to the pair's emission slot, so a record's
//                         partial sums are contiguous.
//   8. record-grad kernel per record: reduce its contiguous partials in order
//                         and apply the chain rule to the 11 parameters.
//   9. view-sum kernel    per Gaussian: sum its records over views in order.
#include "splat_math.h"

namespace fgs {
namespace {

constexpr int kTS = 16;          // tile side in pixels
constexpr int kWave = 64;        // lanes per wave (gfx9 wave64)
constexpr int kRows = 4;         // pixels per lane in the forward (a column of 4)

// Tile span of [c - r, c + r] for pixel centres at j + 1/2. Plain float32
// subtractions and floor: the same decision the integer reference takes.
__device__ __forceinline__ void tile_span(float c, float r, int n_tiles, int &t0, int &t1) {
#pragma clang fp contract(off)
  const float lim = 16777216.f;
  float lo = (c - r) - 0.5f;
  float hi = (c + r) - 0.5f;
  lo = fminf(fmaxf(lo, -lim), lim);
  hi = fminf(fmaxf(hi, -lim), lim);
  const int jlo = static_cast<int>(floorf(lo));
  const int jhi = static_cast<int>(floorf(hi));
  t0 = max(jlo >> 4, 0);
  t1 = min(jhi >> 4, n_tiles - 1);
}

__global__ void zero_u64_kernel(unsigned long long *p) { *p = 0ull; }

// Record r = v_local * n + i of one (view, Gaussian) pair. Returns its tile count.
__device__ __forceinline__ uint32_t record_one(const fgs_gaussians &g, const GeomDev &G, int64_t i,
                                               int v_local, float2 *__restrict__ xy,
                                               float4 *__restrict__ conic_w, float2 *__restrict__ radii,
                                               ushort4 *__restrict__ rect, uint32_t *__restrict__ count) {
  const int64_t r = int64_t(v_local) * g.n + i;
  GaussParams P;
  load_gauss(g, i, P);
  ViewFrame F;
  make_frame(G, G.view_begin + v_local, F);
  Splat S;
  splat_forward(P, F, G, S);
  if (!S.ok) {
    xy[r] = make_float2(0.f, 0.f);
    conic_w[r] = make_float4(0.f, 0.f, 0.f, 0.f);
    radii[r] = make_float2(0.f, 0.f);
    rect[r] = make_ushort4(1, 1, 0, 0);
    count[r] = 0;
    return 0;
  }
  const float ru = G.kappa * sqrtf(S.a);
  const float rv = G.kappa * sqrtf(S.c);
  int x0, x1, y0, y1;
  tile_span(S.u, ru, G.tiles_x, x0, x1);
  tile_span(S.v, rv, G.tiles_y, y0, y1);
  const bool empty = (x0 > x1) || (y0 > y1);
  const float k = -0.5f * kLog2e;
  xy[r] = make_float2(S.u, S.v);
  conic_w[r] = make_float4(k * S.C00, 2.f * k * S.C01, k * S.C11, S.w);
  radii[r] = make_float2(ru, rv);
  if (empty) {
    rect[r] = make_ushort4(1, 1, 0, 0);
    count[r] = 0;
    return 0;
  }
  rect[r] = make_ushort4(x0, y0, x1, y1);
  const uint32_t cnt = uint32_t(x1 - x0 + 1) * uint32_t(y1 - y0 + 1);
  count[r] = cnt;
  return cnt;
}

__global__ __launch_bounds__(256) void record_kernel(fgs_gaussians g, GeomDev G, float2 *__restrict__ xy,
                                                     float4 *__restrict__ conic_w,
                                                     float2 *__restrict__ radii,
                                                     ushort4 *__restrict__ rect,
                                                     uint32_t *__restrict__ count,
                                                     unsigned long long *__restrict__ total64) {
  const int64_t i = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  uint32_t cnt = 0;
  if (i < g.n) cnt = record_one(g, G, i, int(blockIdx.y), xy, conic_w, radii, rect, count);
  // 64-bit pair total (detects a 32-bit scan overflow): one atomic per wave
  unsigned long long w = cnt;
  for (int d = 32; d > 0; d >>= 1) w += __shfl_xor(w, d, 64);
  if ((threadIdx.x & 63) == 0 && w) atomicAdd(total64, w);
}

__global__ __launch_bounds__(256) void emit_kernel(uint64_t R, int64_t n, int tiles_x, int tpv,
                                                   const ushort4 *__restrict__ rect,
                                                   const uint32_t *__restrict__ offset,
                                                   uint32_t *__restrict__ keys,
                                                   uint32_t *__restrict__ vals) {
  const uint64_t r = uint64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (r >= R) return;
  uint32_t o = offset[r];
  const uint32_t end = offset[r + 1];
  if (o == end) return;
  const ushort4 rc = rect[r];
  const uint32_t base = uint32_t(r / uint64_t(n)) * uint32_t(tpv);
  for (int ty = rc.y; ty <= rc.w; ++ty)
    for (int tx = rc.x; tx <= rc.z; ++tx) {
      keys[o] = base + uint32_t(ty * tiles_x + tx);
      vals[o] = uint32_t(r);
      ++o;
    }
}

// start[t] = first sorted position whose key is >= t, for t in [0, T].
__global__ __launch_bounds__(256) void ranges_kernel(const uint32_t *__restrict__ skeys, uint64_t K,
                                                     uint32_t T, uint32_t *__restrict__ start) {
  const uint64_t k = uint64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (k > K) return;
  const int64_t prev = (k == 0) ? -1 : int64_t(skeys[k - 1]);
  const int64_t cur = (k == K) ? int64_t(T) : int64_t(skeys[k]);
  for (int64_t t = prev + 1; t <= cur; ++t) start[t] = uint32_t(k);
}

// kCount = true: instead of the image, count the (pixel, Gaussian) pairs in
// the support whose pixel lies on the detector (the algorithmic work).
template <bool kCount>
__global__ __launch_bounds__(kWave) void splat_fwd_kernel(const uint32_t *__restrict__ start,
                                                          const uint32_t *__restrict__ svals,
                                                          const float2 *__restrict__ xy,
                                                          const float4 *__restrict__ conic_w,
                                                          int tiles_x, int tpv, int W, int H,
                                                          float thr, float *__restrict__ img,
                                                          unsigned long long *__restrict__ counter) {
  __shared__ float4 s_cw[kWave];
  __shared__ float2 s_xy[kWave];
  const uint32_t tile = blockIdx.x;
  const uint32_t v_local = tile / uint32_t(tpv);
  const uint32_t t = tile - v_local * uint32_t(tpv);
  const int ty = int(t) / tiles_x;
  const int tx = int(t) - ty * tiles_x;
  const int lane = threadIdx.x;
  const int col = lane & (kTS - 1);
  const int row0 = (lane >> 4) * kRows;
  const float px = float(tx * kTS + col) + 0.5f;
  const float py = float(ty * kTS + row0) + 0.5f;
  float acc[kRows];
#pragma unroll
  for (int k = 0; k < kRows; ++k) acc[k] = 0.f;
  const uint32_t b0 = start[tile], e = start[tile + 1];
  for (uint32_t b = b0; b < e; b += kWave) {
    const uint32_t m = min(uint32_t(kWave), e - b);
    if (uint32_t(lane) < m) {
      const uint32_t r = svals[b + lane];
      s_cw[lane] = conic_w[r];
      s_xy[lane] = xy[r];
    }
    __syncthreads();
    for (uint32_t j = 0; j < m; ++j) {
      const float4 c = s_cw[j];
      const float2 q = s_xy[j];
      const float dx = px - q.x;
      const float dy = py - q.y;
      const float A = c.x * dx * dx;
      const float B = c.y * dx;
#pragma unroll
      for (int k = 0; k < kRows; ++k) {
        const float d = dy + float(k);
        const float arg = fmaf(d, fmaf(c.z, d, B), A);
        if (kCount) {
          acc[k] += (arg >= thr) ? 1.f : 0.f;
        } else {
          const float ex = __builtin_amdgcn_exp2f(arg);
          acc[k] += (arg >= thr) ? c.w * ex : 0.f;
        }
      }
    }
    __syncthreads();
  }
  const int x = tx * kTS + col;
  if (kCount) {
    unsigned long long n = 0;
#pragma unroll
    for (int k = 0; k < kRows; ++k) {
      const int y = ty * kTS + row0 + k;
      if (x < W && y < H) n += static_cast<unsigned long long>(acc[k]);
    }
    for (int d = 32; d > 0; d >>= 1) n += __shfl_xor(n, d, 64);
    if (lane == 0 && n) atomicAdd(counter, n);
    return;
  }
  float *out = img + uint64_t(v_local) * uint64_t(W) * uint64_t(H);
#pragma unroll
  for (int k = 0; k < kRows; ++k) {
    const int y = ty * kTS + row0 + k;
    if (x < W && y < H) out[uint64_t(y) * W + x] = acc[k];
  }
}

__global__ __launch_bounds__(kWave) void splat_bwd_kernel(
    const uint32_t *__restrict__ start, const uint32_t *__restrict__ svals,
    const float2 *__restrict__ xy, const float4 *__restrict__ conic_w,
    const ushort4 *__restrict__ rect, const uint32_t *__restrict__ offset, int tiles_x, int tpv,
    int W, int H, float thr, const float *__restrict__ gimg, float2 *__restrict__ partials) {
  __shared__ float s_g[kTS * kTS];
  const uint32_t tile = blockIdx.x;
  const uint32_t v_local = tile / uint32_t(tpv);
  const uint32_t t = tile - v_local * uint32_t(tpv);
  const int ty = int(t) / tiles_x;
  const int tx = int(t) - ty * tiles_x;
  const int lane = threadIdx.x;
  const float *gv = gimg + uint64_t(v_local) * uint64_t(W) * uint64_t(H);
  for (int p = lane; p < kTS * kTS; p += kWave) {
    const int x = tx * kTS + (p & (kTS - 1));
    const int y = ty * kTS + (p >> 4);
    s_g[p] = (x < W && y < H) ? gv[uint64_t(y) * W + x] : 0.f;
  }
  __syncthreads();
  const uint32_t b0 = start[tile], e = start[tile + 1];
  const float ox = float(tx * kTS) + 0.5f, oy = float(ty * kTS) + 0.5f;
  for (uint32_t b = b0; b < e; b += kWave) {
    const uint32_t k = b + lane;
    const bool active = k < e;
    float4 c = make_float4(0.f, 0.f, 0.f, 0.f);
    float2 q = make_float2(0.f, 0.f);
    uint32_t r = 0;
    if (active) {
      r = svals[k];
      c = conic_w[r];
      q = xy[r];
    }
    // pixel (col, row) of the tile sits at (col - qx, row - qy) from the centre
    const float qx = q.x - ox, qy = q.y - oy;
    float S0 = 0.f, Sx = 0.f, Sy = 0.f, Sxx = 0.f, Sxy = 0.f, Syy = 0.f;
    for (int row = 0; row < kTS; ++row) {
      const float dy = float(row) - qy;
      const float B = c.y * dy;
      const float Cc = c.z * dy * dy;
      float R0 = 0.f, RX = 0.f, RXX = 0.f;
#pragma unroll
      for (int col = 0; col < kTS; ++col) {
        const float dx = float(col) - qx;
        const float arg = fmaf(dx, fmaf(c.x, dx, B), Cc);
        const float ex = __builtin_amdgcn_exp2f(arg);
        const float ge = (arg >= thr) ? s_g[row * kTS + col] * ex : 0.f;
        R0 += ge;
        const float gx = ge * dx;
        RX += gx;
        RXX = fmaf(gx, dx, RXX);
      }
      S0 += R0;
      Sx += RX;
      Sy = fmaf(R0, dy, Sy);
      Sxx += RXX;
      Sxy = fmaf(RX, dy, Sxy);
      Syy = fmaf(R0 * dy, dy, Syy);
    }
    if (active) {
      const ushort4 rc = rect[r];
      const uint32_t j = uint32_t(ty - rc.y) * uint32_t(rc.z - rc.x + 1) + uint32_t(tx - rc.x);
      const uint64_t p = uint64_t(offset[r]) + j;
      partials[3 * p + 0] = make_float2(S0, Sx);
      partials[3 * p + 1] = make_float2(Sy, Sxx);
      partials[3 * p + 2] = make_float2(Sxy, Syy);
    }
  }
}

__global__ __launch_bounds__(256) void record_grad_kernel(fgs_gaussians g, GeomDev G,
                                                          const uint32_t *__restrict__ offset,
                                                          const float2 *__restrict__ partials,
                                                          uint64_t R, float *__restrict__ grad_rec) {
  const int64_t i = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (i >= g.n) return;
  const int v_local = blockIdx.y;
  const uint64_t r = uint64_t(v_local) * uint64_t(g.n) + uint64_t(i);
  const uint32_t o = offset[r], end = offset[r + 1];
  float out[11];
  if (o == end) {
#pragma unroll
    for (int c = 0; c < 11; ++c) grad_rec[uint64_t(c) * R + r] = 0.f;
    return;
  }
  float sums[6] = {0.f, 0.f, 0.f, 0.f, 0.f, 0.f};
  for (uint32_t p = o; p < end; ++p) {
    const float2 a = partials[3 * uint64_t(p) + 0];
    const float2 b = partials[3 * uint64_t(p) + 1];
    const float2 c = partials[3 * uint64_t(p) + 2];
    sums[0] += a.x; sums[1] += a.y; sums[2] += b.x;
    sums[3] += b.y; sums[4] += c.x; sums[5] += c.y;
  }
  GaussParams P;
  load_gauss(g, i, P);
  ViewFrame F;
  make_frame(G, G.view_begin + v_local, F);
  Splat S;
  splat_forward(P, F, G, S);
  if (!S.ok) {
#pragma unroll
    for (int c = 0; c < 11; ++c) grad_rec[uint64_t(c) * R + r] = 0.f;
    return;
  }
  // moments are relative to the pixel coordinate frame: the sums use
  // (pixel - centre); the kernel's pre-scaled conic is undone here
  splat_backward(P, F, G, S, sums, out);
#pragma unroll
  for (int c = 0; c < 11; ++c) grad_rec[uint64_t(c) * R + r] = out[c];
}

__global__ __launch_bounds__(256) void view_sum_kernel(int64_t n, int views,
                                                       const float *__restrict__ grad_rec,
                                                       fgs_gaussian_grads out) {
  const int64_t i = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const uint64_t R = uint64_t(views) * uint64_t(n);
  float acc[11];
#pragma unroll
  for (int c = 0; c < 11; ++c) acc[c] = 0.f;
  for (int v = 0; v < views; ++v) {
    const uint64_t r = uint64_t(v) * uint64_t(n) + uint64_t(i);
#pragma unroll
    for (int c = 0; c < 11; ++c) acc[c] += grad_rec[uint64_t(c) * R + r];
  }
  out.mean[i] = acc[0]; out.mean[n + i] = acc[1]; out.mean[2 * n + i] = acc[2];
  out.log_scale[i] = acc[3]; out.log_scale[n + i] = acc[4]; out.log_scale[2 * n + i] = acc[5];
  out.quat[i] = acc[6]; out.quat[n + i] = acc[7]; out.quat[2 * n + i] = acc[8]; out.quat[3 * n + i] = acc[9];
  out.density[i] = acc[10];
}

// ------------------------------------------------------------------ host

struct RastLayout {
  uint64_t R, T, K;
  // byte offsets
  uint64_t total64, xy, radii, rect, offset, conic, scan_scratch, start, grad_rec;
  uint64_t fixed_end;
  uint64_t keys, vals, keys_alt, vals_alt, sort_scratch, partials;
  uint64_t total;
  bool sorted_in_alt;
};

RastLayout rast_layout(uint64_t R, uint64_t T, uint64_t K) {
  RastLayout L{};
  L.R = R;
  L.T = T;
  L.K = K;
  Carver c(nullptr);
  c.take<unsigned long long>(1, &L.total64);
  c.take<float2>(R, &L.xy);
  c.take<float2>(R, &L.radii);
  c.take<ushort4>(R, &L.rect);
  c.take<uint32_t>(R + 1, &L.offset);
  c.take<float4>(R, &L.conic);
  c.take<uint32_t>(scan_scratch_words(R), &L.scan_scratch);
  c.take<uint32_t>(T + 1, &L.start);
  c.take<float>(11 * R, &L.grad_rec);
  L.fixed_end = c.used;
  c.take<uint32_t>(K, &L.keys);
  c.take<uint32_t>(K, &L.vals);
  c.take<uint32_t>(K, &L.keys_alt);
  c.take<uint32_t>(K, &L.vals_alt);
  c.take<uint32_t>(sort_scratch_words(K), &L.sort_scratch);
  c.take<float>(6 * K, &L.partials);
  L.total = c.used;
  const int bits = bits_for(T);
  const int passes = (K > 1 && bits > 0) ? (bits + 8) / 9 : 0;
  L.sorted_in_alt = (passes & 1) != 0;
  return L;
}

struct TileGrid {
  int tiles_x, tiles_y, tpv;
};

TileGrid tile_grid(int det_w, int det_h) {
  TileGrid t;
  t.tiles_x = (det_w + kTS - 1) / kTS;
  t.tiles_y = (det_h + kTS - 1) / kTS;
  t.tpv = t.tiles_x * t.tiles_y;
  return t;
}

template <typename T>
T *at(void *base, uint64_t off) {
  return reinterpret_cast<T *>(static_cast<char *>(base) + off);
}

int validate(const fgs_gaussians *g, const fgs_geom *geom, int32_t view_begin, int32_t view_count,
             const fgs_opts *o, fgs_workspace *ws) {
  if (!g || !geom || !o || !ws) return fail(FGS_E_INVALID, "null argument");
  if (g->n <= 0 || !g->mean || !g->log_scale || !g->quat || !g->density)
    return fail(FGS_E_INVALID, "invalid Gaussians");
  if (g->n > 0x7fffffff) return fail(FGS_E_UNSUPPORTED, "more than 2^31 Gaussians");
  if (geom->mode != FGS_CONE && geom->mode != FGS_PARALLEL) return fail(FGS_E_INVALID, "geometry mode");
  if (!geom->angles || geom->n_views <= 0) return fail(FGS_E_INVALID, "angles");
  if (geom->det_w <= 0 || geom->det_h <= 0 || geom->det_w > 65535 * kTS || geom->det_h > 65535 * kTS)
    return fail(FGS_E_INVALID, "detector size");
  if (!(geom->pitch_u > 0.f) || !(geom->pitch_v > 0.f)) return fail(FGS_E_INVALID, "pitch");
  if (geom->mode == FGS_CONE && (!(geom->sdd > 0.f) || !(geom->sod > 0.f)))
    return fail(FGS_E_INVALID, "sod/sdd");
  if (view_count <= 0 || view_begin < 0 || int64_t(view_begin) + view_count > geom->n_views)
    return fail(FGS_E_INVALID, "view range");
  if (!(o->kappa > 0.f)) return fail(FGS_E_INVALID, "kappa must be > 0");
  return FGS_OK;
}

GeomDev make_geom_dev(const fgs_geom *geom, const fgs_opts *o, int view_begin, const TileGrid &L) {
  GeomDev G{};
  G.mode = geom->mode;
  G.det_w = geom->det_w;
  G.det_h = geom->det_h;
  G.tiles_x = L.tiles_x;
  G.tiles_y = L.tiles_y;
  G.view_begin = view_begin;
  G.sod = geom->sod;
  if (geom->mode == FGS_CONE) {
    G.fu = geom->sdd / geom->pitch_u;
    G.fv = geom->sdd / geom->pitch_v;
  } else {
    G.fu = 1.f / geom->pitch_u;
    G.fv = 1.f / geom->pitch_v;
  }
  G.cu = 0.5f * float(geom->det_w) + geom->off_u;
  G.cv = 0.5f * float(geom->det_h) + geom->off_v;
  G.near_plane = o->near_plane;
  G.kappa = o->kappa;
  G.angles = geom->angles;
  return G;
}

// Steps 1-5. On success the workspace holds records, sorted lists and tile
// starts; *Lout describes them.
int build_lists(const fgs_gaussians *g, const fgs_geom *geom, int32_t view_begin, int32_t view_count,
                const fgs_opts *o, fgs_workspace *ws, hipStream_t s, RastLayout *Lout) {
  const uint64_t R = uint64_t(view_count) * uint64_t(g->n);
  const TileGrid tg = tile_grid(geom->det_w, geom->det_h);
  const uint64_t T = uint64_t(view_count) * uint64_t(tg.tpv);
  if (T >= 0xffffffffull || R >= 0xffffffffull) return fail(FGS_E_UNSUPPORTED, "too many tiles or records in one call");
  RastLayout L = rast_layout(R, T, 0);
  ws->kind = 0;
  if (!ws->ptr || ws->bytes < L.fixed_end + (uint64_t(1) << 20)) {
    ws->needed = L.fixed_end + (uint64_t(64) << 20);
    return fail(FGS_E_CAPACITY, "workspace too small for the per-record arrays");
  }
  GeomDev G = make_geom_dev(geom, o, view_begin, tg);
  void *b = ws->ptr;
  unsigned long long *total64 = at<unsigned long long>(b, L.total64);
  zero_u64_kernel<<<1, 1, 0, s>>>(total64);
  FGS_LAUNCH_CHECK("zero_u64_kernel");
  dim3 rgrid(grid_for(uint64_t(g->n), 256), unsigned(view_count));
  record_kernel<<<rgrid, 256, 0, s>>>(*g, G, at<float2>(b, L.xy), at<float4>(b, L.conic),
                                      at<float2>(b, L.radii), at<ushort4>(b, L.rect),
                                      at<uint32_t>(b, L.offset), total64);
  FGS_LAUNCH_CHECK("record_kernel");
  int st = exclusive_scan_u32(at<uint32_t>(b, L.offset), R, at<uint32_t>(b, L.scan_scratch), s);
  if (st != FGS_OK) return st;
  unsigned long long K64 = 0;
  FGS_HIP(hipMemcpyAsync(&K64, total64, sizeof(K64), hipMemcpyDeviceToHost, s));
  FGS_HIP(hipStreamSynchronize(s));
  if (K64 >= 0xffffffffull)
    return fail(FGS_E_UNSUPPORTED, "more than 2^32 (tile, Gaussian) pairs in one call; split the views");
  const uint64_t K = K64;
  L = rast_layout(R, T, K);
  ws->needed = L.total;
  ws->n_pairs = K;
  ws->n_records = R;
  ws->n_tiles = T;
  if (ws->bytes < L.total) return fail(FGS_E_CAPACITY, "workspace too small for the tile lists");
  if (K > 0) {
    emit_kernel<<<grid_for(R, 256), 256, 0, s>>>(R, g->n, tg.tiles_x, tg.tpv, at<ushort4>(b, L.rect),
                                                  at<uint32_t>(b, L.offset), at<uint32_t>(b, L.keys),
                                                  at<uint32_t>(b, L.vals));
    FGS_LAUNCH_CHECK("emit_kernel");
  }
  uint32_t *sk, *sv;
  st = radix_sort_pairs(at<uint32_t>(b, L.keys), at<uint32_t>(b, L.vals), at<uint32_t>(b, L.keys_alt),
                        at<uint32_t>(b, L.vals_alt), K, bits_for(T), at<uint32_t>(b, L.sort_scratch),
                        &sk, &sv, s);
  if (st != FGS_OK) return st;
  ranges_kernel<<<grid_for(K + 1, 256), 256, 0, s>>>(sk, K, uint32_t(T), at<uint32_t>(b, L.start));
  FGS_LAUNCH_CHECK("ranges_kernel");
  ws->kind = 1;
  *Lout = L;
  return FGS_OK;
}

}  // namespace

int rast_binning_layout(const fgs_workspace *ws, uint64_t off[9], uint64_t counts[3]);

}  // namespace fgs

using namespace fgs;

extern "C" int fgs_project_views_fwd(const fgs_gaussians *g, const fgs_geom *geom, int32_t view_begin,
                                     int32_t view_count, const fgs_opts *opts, float *img,
                                     fgs_workspace *ws, void *stream) {
  int st = validate(g, geom, view_begin, view_count, opts, ws);
  if (st != FGS_OK) return st;
  if (!img) return fail(FGS_E_INVALID, "null image");
  hipStream_t s = static_cast<hipStream_t>(stream);
  RastLayout L;
  st = build_lists(g, geom, view_begin, view_count, opts, ws, s, &L);
  if (st != FGS_OK) return st;
  void *b = ws->ptr;
  const uint32_t *sv = at<uint32_t>(b, L.sorted_in_alt ? L.vals_alt : L.vals);
  const float thr = -0.5f * kLog2e * opts->kappa * opts->kappa;
  const TileGrid tg = tile_grid(geom->det_w, geom->det_h);
  hipEvent_t *ev = static_cast<hipEvent_t *>(opts->events);
  if (ev) FGS_HIP(hipEventRecord(ev[0], s));
  splat_fwd_kernel<false><<<unsigned(L.T), kWave, 0, s>>>(at<uint32_t>(b, L.start), sv, at<float2>(b, L.xy),
                                                          at<float4>(b, L.conic), tg.tiles_x, tg.tpv,
                                                          geom->det_w, geom->det_h, thr, img, nullptr);
  FGS_LAUNCH_CHECK("splat_fwd_kernel");
  if (ev) FGS_HIP(hipEventRecord(ev[1], s));
  return FGS_OK;
}

extern "C" int fgs_project_views_support(const fgs_gaussians *g, const fgs_geom *geom, int32_t view_begin,
                                         int32_t view_count, const fgs_opts *opts, uint64_t *out,
                                         fgs_workspace *ws, void *stream) {
  int st = validate(g, geom, view_begin, view_count, opts, ws);
  if (st != FGS_OK) return st;
  if (!out) return fail(FGS_E_INVALID, "null output");
  hipStream_t s = static_cast<hipStream_t>(stream);
  RastLayout L;
  st = build_lists(g, geom, view_begin, view_count, opts, ws, s, &L);
  if (st != FGS_OK) return st;
  void *b = ws->ptr;
  unsigned long long *cnt = reinterpret_cast<unsigned long long *>(out);
  zero_u64_kernel<<<1, 1, 0, s>>>(cnt);
  FGS_LAUNCH_CHECK("zero_u64_kernel");
  const uint32_t *sv = at<uint32_t>(b, L.sorted_in_alt ? L.vals_alt : L.vals);
  const float thr = -0.5f * kLog2e * opts->kappa * opts->kappa;
  const TileGrid tg = tile_grid(geom->det_w, geom->det_h);
  splat_fwd_kernel<true><<<unsigned(L.T), kWave, 0, s>>>(at<uint32_t>(b, L.start), sv, at<float2>(b, L.xy),
                                                         at<float4>(b, L.conic), tg.tiles_x, tg.tpv,
                                                         geom->det_w, geom->det_h, thr, nullptr, cnt);
  FGS_LAUNCH_CHECK("splat_fwd_kernel<count>");
  return FGS_OK;
}

extern "C" int fgs_project_views_bwd(const fgs_gaussians *g, const fgs_geom *geom, int32_t view_begin,
                                     int32_t view_count, const fgs_opts *opts, const float *grad_img,
                                     fgs_gaussian_grads *out, fgs_workspace *ws, void *stream) {
  int st = validate(g, geom, view_begin, view_count, opts, ws);
  if (st != FGS_OK) return st;
  if (!grad_img || !out || !out->mean || !out->log_scale || !out->quat || !out->density)
    return fail(FGS_E_INVALID, "null gradient buffer");
  hipStream_t s = static_cast<hipStream_t>(stream);
  const uint64_t R = uint64_t(view_count) * uint64_t(g->n);
  RastLayout L;
  if (opts->recompute) {
    st = build_lists(g, geom, view_begin, view_count, opts, ws, s, &L);
    if (st != FGS_OK) return st;
  } else {
    if (ws->kind != 1 || ws->n_records != R || !ws->ptr)
      return fail(FGS_E_INVALID, "workspace does not hold this call's rasterizer lists");
    const uint64_t T = uint64_t(view_count) * uint64_t(tile_grid(geom->det_w, geom->det_h).tpv);
    L = rast_layout(R, T, ws->n_pairs);
    if (T != ws->n_tiles || ws->bytes < L.total)
      return fail(FGS_E_INVALID, "workspace lists do not match this call");
  }
  void *b = ws->ptr;
  const TileGrid tg = tile_grid(geom->det_w, geom->det_h);
  GeomDev G = make_geom_dev(geom, opts, view_begin, tg);
  const uint32_t *sv = at<uint32_t>(b, L.sorted_in_alt ? L.vals_alt : L.vals);
  const float thr = -0.5f * kLog2e * opts->kappa * opts->kappa;
  hipEvent_t *ev = static_cast<hipEvent_t *>(opts->events);
  if (ev) FGS_HIP(hipEventRecord(ev[0], s));
  if (L.K > 0) {
    splat_bwd_kernel<<<unsigned(L.T), kWave, 0, s>>>(
        at<uint32_t>(b, L.start), sv, at<float2>(b, L.xy), at<float4>(b, L.conic),
        at<ushort4>(b, L.rect), at<uint32_t>(b, L.offset), tg.tiles_x, tg.tpv, geom->det_w, geom->det_h,
        thr, grad_img, at<float2>(b, L.partials));
    FGS_LAUNCH_CHECK("splat_bwd_kernel");
  }
  if (ev) FGS_HIP(hipEventRecord(ev[1], s));
  dim3 rgrid(grid_for(uint64_t(g->n), 256), unsigned(view_count));
  record_grad_kernel<<<rgrid, 256, 0, s>>>(*g, G, at<uint32_t>(b, L.offset), at<float2>(b, L.partials), R,
                                           at<float>(b, L.grad_rec));
  FGS_LAUNCH_CHECK("record_grad_kernel");
  view_sum_kernel<<<grid_for(uint64_t(g->n), 256), 256, 0, s>>>(g->n, view_count, at<float>(b, L.grad_rec),
                                                                *out);
  FGS_LAUNCH_CHECK("view_sum_kernel");
  return FGS_OK;
}

namespace fgs {
int rast_binning_layout(const fgs_workspace *ws, uint64_t off[9], uint64_t counts[3]) {
  RastLayout L = rast_layout(ws->n_records, ws->n_tiles, ws->n_pairs);
  off[0] = L.xy;
  off[1] = L.radii;
  off[2] = L.rect;
  off[3] = L.offset;
  off[4] = L.sorted_in_alt ? L.keys : L.keys_alt;
  off[5] = L.sorted_in_alt ? L.vals : L.vals_alt;
  off[6] = L.sorted_in_alt ? L.keys_alt : L.keys;
  off[7] = L.sorted_in_alt ? L.vals_alt : L.vals;
  off[8] = L.start;
  counts[0] = L.R;
  counts[1] = L.K;
  counts[2] = L.T;
  return FGS_OK;
}
}  // namespace fgs
