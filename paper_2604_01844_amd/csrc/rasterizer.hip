// X-ray rasterizer (Eq. 3-4, Sec. 3.2; accelerations of Sec. 3.5) for gfx950.
//
// Forward, per call over a batch of views:
//   1. record kernel      one thread per (view, Gaussian): splat centre,
//                         pre-scaled conic and w = rho mu packed in one
//                         32-byte line with the pair-slot addressing, support
//                         half-extents, axis-aligned tile rectangle, count.
//   2. exclusive scan     counts -> key offsets (one readback of the total).
//   3. emit kernel        keys (view << tile_bits | tile) and values
//                         (record index), row-major inside each rectangle;
//                         completes the record's slot base. Records are
//                         view-major, so the emitted keys already ascend in
//                         the view field.
//   4. radix sort         stable, over the tile field only (two passes of
//                         at most 7 bits for up to 16384 tiles per view):
//                         with the input already in view order this orders
//                         the pairs by (tile, view), each tile's list in
//                         ascending Gaussian index; no depth key (the sum is
//                         order-free).
//   5. ranges kernel      per-(view, tile) [start, end) by boundary detection.
//   6. splat kernel       one 64-lane wave per 16x16 tile, up to 16 tiles
//                         per workgroup; batches of 64 records staged in LDS;
//                         each record is tested against the tile's four 8x8
//                         quadrants and a 16-lane group walks one quadrant's
//                         list, each lane a column of 4 pixels; the Gaussian
//                         factor is one v_exp_f32 of a pre-scaled quadratic
//                         form; support test d^2 <= k^2 (skipped for
//                         quadrants entirely inside the support when
//                         Gaussians span many tiles).
// Backward (per-Gaussian formulation, Sec. 3.5):
//   7. splat-grad kernel  same tiling and quadrant lists; one lane per
//                         (quadrant, Gaussian) pair sums over the quadrant's
//                         64 pixels (dL/dI from LDS) the six moments
//                         sum g e {1, dx, dy, dx^2, dx dy, dy^2}; the lane
//                         that loaded the record gathers its quadrants'
//                         partials by wavefront permutes, in quadrant order,
//                         and writes the pair's sums to its emission slot (32
//                         bytes), so a record's partial sums are contiguous.
//                         No atomics.
//   8. record-grad kernel per record: reduce its contiguous partials in order
//                         and apply the chain rule to the 11 parameters.
//   9. view-sum kernel    per Gaussian: sum its records over views in order.
#include "exact_math.h"

namespace fgs {
namespace {

constexpr int kTS = 16;          // tile side in pixels
constexpr int kWave = 64;        // lanes per wave (gfx9 wave64)
constexpr int kRows = 4;         // pixels per lane (a column of 4): ray-exact forward, per-pixel ablation
constexpr int kFwdRows = 8;      // pixels per lane in the splat forward (a quadrant column)
// The quadrant culling test keeps pairs whose exponent reaches thr * kCullSlack
// (a Mahalanobis radius 0.05% beyond the support), a superset of the per-pixel test.
constexpr float kCullSlack = 1.001f;

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

constexpr float kLn2 = 0.6931471805599453f;

// Support threshold of one record on the pre-scaled exponent
// arg = -log2(e)/2 d^2: thr = -log2(e)/2 kappa^2, raised to log2(tau / w) by
// the density-aware support (Sec. 3.5, boxes that also take the density into
// account: d^2 <= min(kappa^2, 2 ln(w / tau)), i.e. the pair's contribution
// w exp(-d^2/2) >= tau). log2_tau = -infinity when tau = 0 (the kappa support).
__device__ __forceinline__ float support_thr(float thr, float log2_tau, float w) {
  return log2_tau > -INFINITY ? fmaxf(thr, log2_tau - __builtin_amdgcn_logf(w)) : thr;
}

// Widest digit of the rasterizer's sort passes over the tile field. Narrow
// digits keep the per-block histograms small and the output runs long;
// measured on MI355X, two 5-bit passes (1024 tiles per view) beat one 10-bit
// pass by ~0.3 ms per standard-scan step, and two 7-bit passes (16384 tiles)
// beat three 5-bit ones.
constexpr int kRastSortBits = 7;
// Up to this many pairs (a single view or a few) the tile field, at most 10
// bits, is sorted in one pass: with few keys per workgroup-tile the second
// pass's histogram, scan and scatter launches cost more than the wider
// digit's ranking.
constexpr uint64_t kOnePassKeys = uint64_t(4) << 20;

inline int rast_sort_bits(uint64_t K, int tile_bits) {
  return (K <= kOnePassKeys && tile_bits <= kSortMaxBits) ? kSortMaxBits : kRastSortBits;
}

// What the pixel kernels read per (tile, Gaussian) pair, packed in one
// 32-byte line: a = (u, v, pre-scaled conic c00, c01), b = (c11, w, base,
// width), where the pair's emission slot for tile (tx, ty) of the record's
// rectangle is base + ty * width + tx (32-bit wrap-around; base is written
// once the key offsets are known).
struct SplatRec {
  float4 a, b;
};

__global__ void zero_u64_kernel(unsigned long long *p, int n) {
  if (int(threadIdx.x) < n) p[threadIdx.x] = 0ull;
}

// Record r = v_local * n + i of one (view, Gaussian) pair. Returns its tile count.
__device__ __forceinline__ uint32_t record_one(const fgs_gaussians &g, const GeomDev &G, int64_t i,
                                               int v_local, float2 *__restrict__ xy,
                                               SplatRec *__restrict__ rec, float2 *__restrict__ radii,
                                               ushort4 *__restrict__ rect, uint32_t *__restrict__ count) {
  const int64_t r = int64_t(v_local) * g.n + i;
  GaussParams P;
  load_gauss(g, i, P);
  ViewFrame F;
  make_frame(G, G.view_begin + v_local, F);
  Splat S;
  splat_forward(P, F, G, S);
  // density-aware support (tau > 0): d^2 <= min(kappa^2, 2 ln(w / tau)), and
  // the tile box is that ellipse's exact box; a splat whose peak w does not
  // exceed tau contributes nothing
  float kap = G.kappa;
  if (S.ok && G.tau > 0.f) {
    if (S.w > G.tau) {
      const float k2t = 2.f * kLn2 * (log2f(S.w) - log2f(G.tau));
      if (k2t < kap * kap) kap = sqrtf(k2t);
    } else {
      S.ok = false;
    }
  }
  if (!S.ok) {
    xy[r] = make_float2(0.f, 0.f);
    rec[r].a = make_float4(0.f, 0.f, 0.f, 0.f);
    rec[r].b = make_float4(0.f, 0.f, 0.f, 0.f);
    radii[r] = make_float2(0.f, 0.f);
    rect[r] = make_ushort4(1, 1, 0, 0);
    count[r] = 0;
    return 0;
  }
  float ru = kap * sqrtf(S.a);
  float rv = kap * sqrtf(S.c);
  if (G.ablate & FGS_ABLATE_SQUARE_BOX) {
    // square of half-side kappa sqrt(lambda_max): the circle bound
    const float h = 0.5f * (S.a - S.c);
    ru = rv = G.kappa * sqrtf(0.5f * (S.a + S.c) + sqrtf(h * h + S.b * S.b));
  }
  int x0, x1, y0, y1;
  tile_span(S.u, ru, G.tiles_x, x0, x1);
  tile_span(S.v, rv, G.tiles_y, y0, y1);
  const bool empty = (x0 > x1) || (y0 > y1);
  const float k = -0.5f * kLog2e;
  xy[r] = make_float2(S.u, S.v);
  rec[r].a = make_float4(S.u, S.v, k * S.C00, 2.f * k * S.C01);
  rec[r].b = make_float4(k * S.C11, S.w, 0.f, __uint_as_float(empty ? 0u : uint32_t(x1 - x0 + 1)));
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

// Ray-exact model: one 64-byte record per (view, Gaussian) pair,
//   a = (u, v, K00, K01), b = (K11, lu, lv, a0), c = (C00, C01, C11, escale),
//   d = (w, base, width, 0), escale = -t2^2 log2(e) / 2, w = rho sqrt(2 pi),
// in the notation of exact_math.h; the pair slot is base + ty * width + tx.
struct ExactRec {
  float4 a, b, c, d;
};

// The tile rectangle of the support ellipse is widened by this factor, so
// FP32 rounding of the box never drops a pixel the per-pixel test keeps.
constexpr float kExactBoxSlack = 1.0005f;

__device__ __forceinline__ uint32_t record_one_exact(const fgs_gaussians &g, const GeomDev &G, int64_t i,
                                                     int v_local, float2 *__restrict__ xy,
                                                     ExactRec *__restrict__ rec, float2 *__restrict__ radii,
                                                     ushort4 *__restrict__ rect, uint32_t *__restrict__ count) {
  const int64_t r = int64_t(v_local) * g.n + i;
  GaussParams P;
  load_gauss(g, i, P);
  ViewFrame F;
  make_frame(G, G.view_begin + v_local, F);
  ExactSplat X;
  exact_forward(P, F, G, X);
  float dcx = 0.f, dcy = 0.f, hx = 0.f, hy = 0.f, cs00, cs01, cs11;
  const bool ok = X.ok && exact_silhouette(X.K00, X.K01, X.K11, X.lu, X.lv, X.a0, X.C00, X.C01, X.C11,
                                           X.t[2] * X.t[2], G.kappa * G.kappa, dcx, dcy, hx, hy, cs00, cs01,
                                           cs11);
  int x0 = 1, x1 = 0, y0 = 1, y1 = 0;
  const float cx = X.u + dcx, cy = X.v + dcy;
  const float ru = hx * kExactBoxSlack, rv = hy * kExactBoxSlack;
  if (ok) {
    tile_span(cx, ru, G.tiles_x, x0, x1);
    tile_span(cy, rv, G.tiles_y, y0, y1);
  }
  const bool empty = !ok || (x0 > x1) || (y0 > y1);
  if (!ok) {
    xy[r] = make_float2(0.f, 0.f);
    radii[r] = make_float2(0.f, 0.f);
    rec[r].a = rec[r].b = rec[r].c = rec[r].d = make_float4(0.f, 0.f, 0.f, 0.f);
  } else {
    xy[r] = make_float2(cx, cy);
    radii[r] = make_float2(ru, rv);
    rec[r].a = make_float4(X.u, X.v, X.K00, X.K01);
    rec[r].b = make_float4(X.K11, X.lu, X.lv, X.a0);
    rec[r].c = make_float4(X.C00, X.C01, X.C11, X.esn * kLog2e);
    rec[r].d = make_float4(X.w, 0.f, __uint_as_float(empty ? 0u : uint32_t(x1 - x0 + 1)), 0.f);
  }
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

template <bool kExact>
__global__ __launch_bounds__(256) void record_kernel(fgs_gaussians g, GeomDev G, float2 *__restrict__ xy,
                                                     void *__restrict__ rec,
                                                     float2 *__restrict__ radii,
                                                     ushort4 *__restrict__ rect,
                                                     uint32_t *__restrict__ count) {
  const int64_t i = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (i >= g.n) return;
  if (kExact)
    record_one_exact(g, G, i, int(blockIdx.y), xy, static_cast<ExactRec *>(rec), radii, rect, count);
  else
    record_one(g, G, i, int(blockIdx.y), xy, static_cast<SplatRec *>(rec), radii, rect, count);
}

// record_bits > 0: one-word lists, keys[q] = tile << record_bits | record
// (the view is the record's, r / n) and no values; else keys[q] = view <<
// tile_bits | tile and vals[q] = the record.
// RPB records per block (kEmitBlock or fewer: calls with few records take
// fewer per block, so that more waves share the keys).
template <int RPB>
__global__ __launch_bounds__(kEmitBlock) void emit_kernel(uint64_t R, int64_t n, int tiles_x, int tile_bits,
                                                          int record_bits, const ushort4 *__restrict__ rect,
                                                          const uint32_t *__restrict__ offset,
                                                          uint32_t *__restrict__ keys,
                                                          uint32_t *__restrict__ vals, float *__restrict__ base_field,
                                                          uint32_t base_stride, const uint32_t *__restrict__ kdev) {
  // nothing to emit: no pairs, or more than the lists were laid out for
  if (kdev[0] == 0u) return;
  static_assert(RPB <= kEmitBlock, "one record per thread at most");
  __shared__ uint32_t s_off[RPB + 1];
  __shared__ ushort4 s_rect[RPB];
  const uint64_t r0 = uint64_t(blockIdx.x) * RPB;
  const int nr = int(min(uint64_t(RPB), R - r0));
  const int t = threadIdx.x;
  if (t < nr) {
    const uint64_t r = r0 + t;
    const uint32_t o = offset[r];
    const ushort4 rc = rect[r];
    s_off[t] = o;
    s_rect[t] = rc;
    if (offset[r + 1] != o) {
      const uint32_t wdt = uint32_t(rc.z) - rc.x + 1u;
      base_field[r * base_stride] = __uint_as_float(o - uint32_t(rc.y) * wdt - uint32_t(rc.x));
    }
  }
  if (t == 0) s_off[nr] = offset[r0 + nr];
  __syncthreads();
  const uint32_t o0 = s_off[0], oe = s_off[nr];
  // each wave writes a contiguous quarter of the block's keys, 64 at a time;
  // a lane finds its first key's record by binary search, then walks forward
  // (its keys ascend, and so do their records)
  constexpr int kEmitWaves = kEmitBlock / 64;
  const int wid = t >> 6, lane = t & 63;
  const uint32_t span = oe - o0, per_wave = (span + kEmitWaves - 1) / kEmitWaves;
  const uint32_t qa = o0 + min(span, uint32_t(wid) * per_wave);
  const uint32_t qb = o0 + min(span, uint32_t(wid + 1) * per_wave);
  int i = -1;
  for (uint32_t q = qa + uint32_t(lane); q < qb; q += 64) {
    if (i < 0)
      i = upper_index(s_off, nr, q);
    else
      while (s_off[i + 1] <= q) ++i;  // s_off[nr] = oe > q ends the walk
    const ushort4 rc = s_rect[i];
    const uint32_t wdt = uint32_t(rc.z) - rc.x + 1u;
    const uint32_t j = q - s_off[i];
    const uint32_t dy = j / wdt;
    const uint64_t r = r0 + i;
    const uint32_t tile = (uint32_t(rc.y) + dy) * uint32_t(tiles_x) + uint32_t(rc.x) + (j - dy * wdt);
    if (record_bits) {
      keys[q] = (tile << record_bits) | uint32_t(r);
    } else {
      keys[q] = (uint32_t(r / uint64_t(n)) << tile_bits) | tile;
      vals[q] = uint32_t(r);
    }
  }
}

__global__ __launch_bounds__(256) void zero_ranges_kernel(uint2 *__restrict__ rng, uint64_t T) {
  const uint64_t t = uint64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (t < T) rng[t] = make_uint2(0u, 0u);
}

// rng[v * tpv + t] = [first, last + 1) of key (v << tile_bits | t) in the
// sorted keys; each key's pairs are contiguous there (tiles without pairs
// keep the empty range the zero kernel wrote).
// A wave takes kRangeItems * 64 consecutive keys, all loads issued first, and
// finds each key's neighbours in the adjacent lanes (across rounds through
// lanes 0 and 63); only the keys just outside its span are loaded twice.
constexpr int kRangeItems = 16;

// One-word lists (record_bits > 0): a word's key is (record / n) <<
// tile_bits | (word >> record_bits).
__device__ __forceinline__ uint32_t list_key(uint32_t w, int record_bits, int tile_bits, uint32_t n) {
  return record_bits ? (((w & ((1u << record_bits) - 1u)) / n) << tile_bits) | (w >> record_bits) : w;
}

// Every tile's range [x, y) of the sorted list, (0, 0) for a tile without
// keys. The list is in (tile, view) order (the sort is on the tile field and
// stable, and records ascend with the view), so a key's rank in that order
// is tile * V + view for V = T / tpv views. The wave holding the first key
// clears the tiles of the ranks before it, the wave holding the last key
// those after it (the grid clears all T when the device holds no keys), and
// the first key of each run those of the ranks between the previous run's
// and its own.
__device__ __forceinline__ uint32_t rank_tile(uint32_t q, uint32_t V, uint32_t tpv) {
  const uint32_t tt = V == 1u ? q : q / V;
  return (q - tt * V) * tpv + tt;
}

__global__ __launch_bounds__(256) void ranges_kernel(const uint32_t *__restrict__ skeys, uint64_t K_cap,
                                                     const uint32_t *__restrict__ kdev, int tile_bits,
                                                     uint32_t tpv, int record_bits, uint32_t n, uint64_t T,
                                                     uint2 *__restrict__ rng) {
  const uint64_t K = min(K_cap, uint64_t(kdev[0]));
  if (K == 0) {
    for (uint64_t t = uint64_t(blockIdx.x) * blockDim.x + threadIdx.x; t < T; t += uint64_t(gridDim.x) * blockDim.x)
      rng[t] = make_uint2(0u, 0u);
    return;
  }
  const uint32_t V = uint32_t(T / tpv);
  const uint32_t tmask = (1u << tile_bits) - 1u;
  const int lane = threadIdx.x & (kWave - 1);
  const uint64_t base = ((uint64_t(blockIdx.x) * blockDim.x + threadIdx.x) >> 6) * uint64_t(kWave * kRangeItems);
  if (base >= K) return;  // uniform over the wave
  uint32_t key[kRangeItems];
#pragma unroll
  for (int j = 0; j < kRangeItems; ++j) {
    const uint64_t k = base + uint64_t(j) * kWave + lane;
    key[j] = k < K ? skeys[k] : 0u;
  }
  const uint64_t after = base + uint64_t(kWave * kRangeItems);
  uint32_t edge_prev = (lane == 0 && base > 0) ? skeys[base - 1] : 0u;
  uint32_t edge_next = (lane == kWave - 1 && after < K) ? skeys[after] : 0u;
  if (record_bits) {
#pragma unroll
    for (int j = 0; j < kRangeItems; ++j) key[j] = list_key(key[j], record_bits, tile_bits, n);
    edge_prev = list_key(edge_prev, record_bits, tile_bits, n);
    edge_next = list_key(edge_next, record_bits, tile_bits, n);
  }
  // the wave of the first key clears the ranks before it, the wave of the
  // last key those after it
  if (base == 0) {
    const uint32_t f = uint32_t(__builtin_amdgcn_readfirstlane(int(key[0])));
    const uint32_t lo = (f & tmask) * V + (f >> tile_bits);
    for (uint32_t q = uint32_t(lane); q < lo; q += kWave) rng[rank_tile(q, V, tpv)] = make_uint2(0u, 0u);
  }
  if (K - 1 - base < uint64_t(kWave * kRangeItems)) {
    const int jl = int((K - 1 - base) / kWave), ll = int((K - 1 - base) % kWave);
    uint32_t l = 0;
#pragma unroll
    for (int j = 0; j < kRangeItems; ++j)
      if (j == jl) l = uint32_t(__builtin_amdgcn_readlane(int(key[j]), ll));
    const uint32_t hi = (l & tmask) * V + (l >> tile_bits) + 1u;
    for (uint32_t q = hi + uint32_t(lane); q < uint32_t(T); q += kWave) rng[rank_tile(q, V, tpv)] = make_uint2(0u, 0u);
  }
#pragma unroll
  for (int j = 0; j < kRangeItems; ++j) {
    const uint64_t k = base + uint64_t(j) * kWave + lane;
    const uint32_t kv = key[j];
    uint32_t prev = __shfl_up(kv, 1, kWave), next = __shfl_down(kv, 1, kWave);
    const uint32_t prev_round = j > 0 ? uint32_t(__builtin_amdgcn_readlane(int(key[j > 0 ? j - 1 : 0]), kWave - 1)) : 0u;
    const uint32_t next_round =
        j + 1 < kRangeItems ? uint32_t(__builtin_amdgcn_readlane(int(key[j + 1 < kRangeItems ? j + 1 : j]), 0)) : 0u;
    if (lane == 0) prev = j > 0 ? prev_round : (base > 0 ? edge_prev : ~kv);
    if (lane == kWave - 1) next = j + 1 < kRangeItems ? next_round : edge_next;
    if (k < K) {
      if (k + 1 == K) next = ~kv;
      const uint32_t tile = (kv >> tile_bits) * tpv + (kv & tmask);
      const uint32_t rank = (kv & tmask) * V + (kv >> tile_bits);
      if (prev != kv) {
        rng[tile].x = uint32_t(k);
        if (k > 0)
          for (uint32_t q = (prev & tmask) * V + (prev >> tile_bits) + 1u; q < rank; ++q)
            rng[rank_tile(q, V, tpv)] = make_uint2(0u, 0u);
      }
      if (next != kv) rng[tile].y = uint32_t(k + 1);
    }
  }
}

// ---------------------------------------------------------------- work units
//
// Calls with few tiles (a single view: 1024 tiles of 512^2) cannot fill the
// chip with one wave per tile, and their list lengths vary widely (on a
// standard-scan view from 0 to about 3,500 keys). Their lists are split into
// contiguous pieces of at least kUnitKeys keys (more when a list would need
// more than kMaxUnits pieces), one wave each, so the units are of nearly
// equal size whatever the spread; an empty tile gets one unit (the forward
// still writes its zero pixels). first[t] is the first unit of tile t
// (first[T] = the number of units), tile[u] the tile of unit u. The forward
// writes each unit's 16 x 16 partial sums to its own slot, and every pixel
// then adds its tile's units in order, so the result is deterministic.
constexpr uint32_t kUnitKeys = 128;
constexpr uint32_t kMaxUnits = 32;

__device__ __forceinline__ uint32_t unit_keys(uint32_t len) {
  const uint32_t per = (len + kMaxUnits - 1) / kMaxUnits;
  return max(kUnitKeys, (per + kWave - 1) / kWave * kWave);
}

__device__ __forceinline__ uint32_t units_of(uint32_t len) {
  return len == 0 ? 1u : (len + unit_keys(len) - 1) / unit_keys(len);
}

// Units of a call, or first == null: a fixed number of strided chunks per tile.
struct Units {
  const uint32_t *first;   // [T + 1]
  const uint32_t *tile;    // [cap]
  uint32_t cap;            // units the launch covers (an upper bound)
};

// Units that T tiles holding K pairs can need: sum over tiles of
// ceil(len / kUnitKeys) + 1 at most.
inline uint64_t units_bound(uint64_t T, uint64_t K) { return T + (K + kUnitKeys - 1) / kUnitKeys; }

// The unit of this wave in a launch over U.cap units, false past the units
// of the call. The launch is sized for the bound, which at a fixed key
// capacity can be twice the units there are; the XCD-aware order is taken
// over the blocks that hold units, so that they spread over all XCDs rather
// than filling the lower ones while the upper ones get the empty blocks.
template <int TPB>
__device__ __forceinline__ bool unit_of_wave(const Units &U, uint32_t n_tiles, int wid, uint32_t &unit) {
  const uint32_t nu = min(U.first[n_tiles], U.cap);
  const uint32_t nb = (nu + uint32_t(TPB) - 1) / uint32_t(TPB);
  if (blockIdx.x >= nb) return false;
  unit = uint32_t(__builtin_amdgcn_readfirstlane(int(xcd_block(blockIdx.x, nb) * uint32_t(TPB) + uint32_t(wid))));
  return unit < nu;
}

// One workgroup of 1024 threads, T <= 8192 tiles (8 per thread).
__global__ __launch_bounds__(1024) void unit_offsets_kernel(const uint2 *__restrict__ rng, uint32_t T, uint32_t cap,
                                                           uint32_t *__restrict__ first, uint32_t *__restrict__ tile) {
  __shared__ uint32_t wsum[16];
  const uint32_t per = (T + 1023u) / 1024u;
  const uint32_t t0 = threadIdx.x * per;
  uint32_t cnt[8];
  uint32_t s = 0;
#pragma unroll
  for (uint32_t j = 0; j < 8; ++j) {
    const uint32_t t = t0 + j;
    cnt[j] = (j < per && t < T) ? units_of(rng[t].y - rng[t].x) : 0u;
    s += cnt[j];
  }
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  uint32_t x = s;
#pragma unroll
  for (int d = 1; d < 64; d <<= 1) {
    const uint32_t y = __shfl_up(x, d, 64);
    if (lane >= d) x += y;
  }
  if (lane == 63) wsum[w] = x;
  __syncthreads();
  uint32_t base = 0, tot = 0;
#pragma unroll
  for (int k = 0; k < 16; ++k) {
    base += k < w ? wsum[k] : 0u;
    tot += wsum[k];
  }
  base += x - s;
  if (threadIdx.x == 0) first[T] = tot;
#pragma unroll
  for (uint32_t j = 0; j < 8; ++j) {
    const uint32_t t = t0 + j;
    if (j < per && t < T) {
      first[t] = base;
      for (uint32_t u = 0; u < cnt[j]; ++u)
        if (base + u < cap) tile[base + u] = t;
      base += cnt[j];
    }
  }
}

// img[v][y][x] = sum over the units u of the pixel's tile, in order, of
// part[u][y % 16][x % 16] (each unit's 16 x 16 partial sums)
__global__ __launch_bounds__(256) void sum_units_kernel(const float *__restrict__ part, const uint32_t *__restrict__ first,
                                                        int tiles_x, int tpv, int W, int H, uint64_t n_img,
                                                        float *__restrict__ img) {
  const uint64_t i = uint64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (i >= n_img) return;
  const uint64_t wh = uint64_t(W) * uint64_t(H);
  const uint32_t v = uint32_t(i / wh);
  const uint32_t p = uint32_t(i - uint64_t(v) * wh);
  const uint32_t y = p / uint32_t(W), x = p - y * uint32_t(W);
  const uint32_t t = v * uint32_t(tpv) + (y / kTS) * uint32_t(tiles_x) + x / kTS;
  const uint32_t lp = (y % kTS) * kTS + (x % kTS);
  const uint32_t u0 = first[t], u1 = first[t + 1];
  const float *q = part + uint64_t(u0) * (kTS * kTS) + lp;
  const uint32_t nu = u1 - u0;
  float acc = q[0];
  // eight loads in flight at a time, added in unit order
  for (uint32_t u = 1; u < nu; u += 8) {
    float x[8];
#pragma unroll
    for (int j = 0; j < 8; ++j) x[j] = u + j < nu ? q[uint64_t(u + j) * (kTS * kTS)] : 0.f;
#pragma unroll
    for (int j = 0; j < 8; ++j)
      if (u + j < nu) acc += x[j];
  }
  img[i] = acc;
}

// ---------------------------------------------------------------- quadrants
//
// Both pixel kernels split a 16x16 tile into four 8x8 quadrants. For every
// (tile, Gaussian) pair of a batch the lane that loads the record tests the
// Gaussian's support ellipse against each quadrant exactly (the smallest
// Mahalanobis distance over the quadrant's pixel centres, below), and the
// wave builds one list of batch slots per quadrant. 16-lane group g then
// works only on quadrant g's list, so pixels outside a Gaussian's support
// ellipse are skipped at 8x8 granularity instead of 16x16.

// Largest value of the pre-scaled form q = c.x dx^2 + c.y dx dy + c.z dy^2
// (q = -log2(e)/2 d^2) over the rectangle [x0, x1] x [y0, y1], relative to
// the centre (u, v): the convex form's minimum of d^2 over a rectangle lies
// on the edge nearest the centre in x or in y, each a clamped 1D minimum.
__device__ __forceinline__ float rect_qmax(const float4 &c, float rx, float ry, float u, float v, float x0,
                                           float x1, float y0, float y1) {
  const float X = fminf(fmaxf(u, x0), x1);
  const float dxa = X - u;
  const float dya = fminf(fmaxf(fmaf(-rx, dxa, v), y0), y1) - v;
  const float qa = fmaf(dxa, fmaf(c.x, dxa, c.y * dya), c.z * dya * dya);
  const float Y = fminf(fmaxf(v, y0), y1);
  const float dyb = Y - v;
  const float dxb = fminf(fmaxf(fmaf(-ry, dyb, u), x0), x1) - u;
  const float qb = fmaf(dxb, fmaf(c.x, dxb, c.y * dyb), c.z * dyb * dyb);
  return fmaxf(qa, qb);
}

// Bit Q set if the support ellipse reaches a pixel centre of quadrant Q of
// the tile whose first pixel centre is (tx0, ty0). thr_cull is a hair below
// the support threshold so the test is a superset of the per-pixel test.
__device__ __forceinline__ uint32_t quad_mask(const float4 &c, float u, float v, float tx0, float ty0,
                                              float thr_cull) {
  const float rx = 0.5f * c.y / c.z;
  const float ry = 0.5f * c.y / c.x;
  uint32_t m = 0;
#pragma unroll
  for (int Q = 0; Q < 4; ++Q) {
    const float x0 = tx0 + float((Q & 1) * 8), y0 = ty0 + float((Q >> 1) * 8);
    if (rect_qmax(c, rx, ry, u, v, x0, x0 + 7.f, y0, y0 + 7.f) >= thr_cull) m |= 1u << Q;
  }
  return m;
}

// Per-quadrant lists of batch slots (slot = lane that loaded the record),
// in slot order. Returns the four list lengths; lane's own positions in the
// lists it belongs to go to pos[Q].
__device__ __forceinline__ void build_quad_lists(uint32_t mask, int lane, uint8_t (*s_list)[kWave],
                                                 int nq[4], int pos[4]) {
  const uint64_t lt = (lane == 0) ? 0ull : (~0ull >> (64 - lane));
#pragma unroll
  for (int Q = 0; Q < 4; ++Q) {
    const bool bit = (mask >> Q) & 1u;
    const uint64_t bal = __ballot(bit);
    pos[Q] = __popcll(bal & lt);
    if (bit) s_list[Q][pos[Q]] = uint8_t(lane);
    nq[Q] = __popcll(bal);
  }
}

// Interior quadrants: every pixel centre of the quadrant lies inside the
// support, so the per-pixel cutoff test can be skipped. The pre-scaled form
// is concave, so its smallest value over the quadrant's pixel-centre square
// is at one of the four corners; thr_int is a hair above the support
// threshold (kInteriorSlack), so FP32 rounding of the per-pixel exponent
// cannot take an interior pixel below thr.
//
// The forward uses it (each 16-lane group takes its quadrant's interior
// pairs first; iterations where all four groups hold interior pairs run
// without the select). The test and the split lists cost a few percent per
// batch, so this pays off only when most pairs are interior, i.e. when
// Gaussians span many tiles: the forward takes the interior path when a call
// averages at least kInteriorKeysPerRecord tiles per record. Measured on
// MI355X: at about 17 tiles per record (50k Gaussians, 512^2 views) 37% of
// the iterations are all-interior and the kernel gets ~8% slower; at about
// 180 (500k Gaussians, 2048^2 views) 77% are, and it gets 7% faster.
constexpr float kInteriorSlack = 0.999f;

// Workgroup size of the splat kernels in large calls. The backward takes 4
// tiles per workgroup always; the forward does when a call averages at least
// kSmallBlockKeysPerTile keys per tile. Measured on MI355X: the backward is
// 2% faster with 4 at about 720 keys per tile (75 views of 512^2, 50k
// Gaussians) and 11% at about 5,700 (10 views of 2048^2, 500k Gaussians);
// the forward is 3% slower with 4 at 720 and 13% faster at 5,700.
constexpr uint64_t kSmallBlockKeysPerTile = 2048;
constexpr uint64_t kInteriorKeysPerRecord = 48;

__device__ __forceinline__ uint32_t quad_interior(const float4 &c, float u, float v, float tx0, float ty0,
                                                  float thr_int) {
  uint32_t m = 0;
#pragma unroll
  for (int Q = 0; Q < 4; ++Q) {
    const float dx0 = tx0 + float((Q & 1) * 8) - u, dy0 = ty0 + float((Q >> 1) * 8) - v;
    float lo = 0.f;
#pragma unroll
    for (int k = 0; k < 4; ++k) {
      const float dx = dx0 + float((k & 1) * 7), dy = dy0 + float((k >> 1) * 7);
      const float a = fmaf(dx, fmaf(c.x, dx, c.y * dy), c.z * dy * dy);
      lo = (k == 0) ? a : fminf(lo, a);
    }
    if (lo >= thr_int) m |= 1u << Q;
  }
  return m;
}

// As build_quad_lists, with each quadrant's interior pairs (imask) first:
// ni[Q] of the nq[Q] entries of list Q need no cutoff test.
__device__ __forceinline__ void build_quad_lists_split(uint32_t mask, uint32_t imask, int lane,
                                                       uint8_t (*s_list)[kWave], int nq[4], int ni[4]) {
  const uint64_t lt = (lane == 0) ? 0ull : (~0ull >> (64 - lane));
#pragma unroll
  for (int Q = 0; Q < 4; ++Q) {
    const bool bi = (imask >> Q) & 1u;
    const uint64_t bal_i = __ballot(bi);
    if (bi) s_list[Q][__popcll(bal_i & lt)] = uint8_t(lane);
    ni[Q] = __popcll(bal_i);
    const bool bb = ((mask & ~imask) >> Q) & 1u;
    const uint64_t bal_b = __ballot(bb);
    if (bb) s_list[Q][ni[Q] + __popcll(bal_b & lt)] = uint8_t(lane);
    nq[Q] = ni[Q] + __popcll(bal_b);
  }
}

// The record indices of the sorted lists. Key/value lists hold them in the
// values array (mask all ones). One-word lists hold (tile << record_bits |
// record) in a single array, sorted on the tile field alone, and the record
// is the word's low record_bits bits.
struct ListRecs {
  const uint32_t *__restrict__ w;
  uint32_t mask;
  __device__ __forceinline__ uint32_t operator[](uint64_t i) const { return w[i] & mask; }
};

// Software pipelining of a tile's record batches: while a batch is being
// evaluated, the next batch's records and the record indices of the one
// after are already in flight, so the two dependent loads (index, then
// record) of a batch overlap the previous batch's arithmetic instead of
// stalling the wave. Lane l holds entry l of its batches. The forward uses
// it (3% faster on 512^2 views); in the backward the eight extra registers
// spilled and it got slower.
template <typename Rec>
struct BatchPrefetch {
  Rec cur, nxt;
  uint32_t idx;  // record index of this lane's entry two batches ahead
  __device__ __forceinline__ static uint32_t count(uint32_t b, uint32_t e) {
    return b < e ? min(uint32_t(kWave), e - b) : 0u;
  }
  // before the loop: records of batch b, indices of batch b + stride
  __device__ __forceinline__ void start(const ListRecs &svals, const Rec *__restrict__ rec, uint32_t b,
                                        uint32_t stride, uint32_t e, int lane) {
    if (uint32_t(lane) < count(b, e)) nxt = rec[svals[b + lane]];
    if (uint32_t(lane) < count(b + stride, e)) idx = svals[b + stride + lane];
  }
  // at the top of the iteration for batch b: cur = batch b's record; issue
  // the loads of batch b + stride (records) and b + 2 stride (indices)
  __device__ __forceinline__ void advance(const ListRecs &svals, const Rec *__restrict__ rec,
                                          uint32_t b, uint32_t stride, uint32_t e, int lane) {
    cur = nxt;
    const uint32_t b1 = b + stride, b2 = b1 + stride;
    if (uint32_t(lane) < count(b1, e)) nxt = rec[idx];
    if (b1 < e && uint32_t(lane) < count(b2, e)) idx = svals[b2 + lane];
  }
};

// Work order of a view's tiles in the backward kernels: strips of four tile
// rows, taken column by column, so consecutive work units (a workgroup's
// tiles) cover 4x4 blocks of tiles instead of pieces of one row.
// Neighbouring tiles have similar list lengths (the waves of a workgroup
// finish closer together) and share records. A bijection of
// [0, tiles_x * tiles_y) for any detector size; the last strip may be lower
// than four rows. Measured on MI355X (standard scan, 75 views of 512^2): the
// splat backward 6% faster; the splat forward 19% slower with the same order,
// so the forward kernels keep row-major order.
__device__ __forceinline__ void tile_of(uint32_t k, int tiles_x, int tiles_y, int &tx, int &ty) {
  const int s = int(k) / (4 * tiles_x);
  const int h = min(4, tiles_y - 4 * s);
  const int r = int(k) - s * 4 * tiles_x;
  tx = r / h;
  ty = 4 * s + (r - tx * h);
}

// Slot kWave of the LDS record arrays holds a record that contributes nothing
// anywhere (zero weight, support far outside every tile).
__device__ __forceinline__ void set_null_record(float4 *s_cw, float2 *s_xy) {
  s_cw[kWave] = make_float4(-1.f, 0.f, -1.f, 0.f);
  s_xy[kWave] = make_float2(-1.0e4f, -1.0e4f);
}

// kCount = true: instead of the image, count the (pixel, Gaussian) pairs in
// the support whose pixel lies on the detector (the algorithmic work).
// kTau: the density-aware support (per-record thresholds, read with each
// pair); without it the pixel loop compares with the kernel argument.
template <bool kCount, bool kInterior, int TPB, bool kTau>
__global__ __launch_bounds__(kWave * TPB) void splat_fwd_kernel(const uint2 *__restrict__ rng,
                                                           const ListRecs svals,
                                                           const SplatRec *__restrict__ rec,
                                                           int tiles_x, int tpv, int W, int H,
                                                           uint32_t n_tiles, int n_chunks, Units U, float thr,
                                                           float log2_tau, int no_cull,
                                                           float *__restrict__ img,
                                                           unsigned long long *__restrict__ counter) {
  // per batch slot: the conic and weight, and (centre, 2 c11, support
  // threshold): one address, the second array at a fixed offset from the first
  __shared__ float4 s_rec_all[TPB][2][kWave + 1];
  __shared__ uint8_t s_list_all[TPB][4][kWave];
  const int wid = threadIdx.x / kWave;
  float4 *s_cw = s_rec_all[wid][0];
  float4 *s_xy = s_rec_all[wid][1];
  uint8_t(*s_list)[kWave] = s_list_all[wid];
  // work unit: a piece of a tile's list (U.first), or (tile, chunk) where
  // chunk c takes batches c, c + n_chunks, ...; each writes its own partial
  // image when there are several per tile
  // everything about the unit is the same across the wave (scalar registers)
  uint32_t unit, tile, chunk, b_first, b_end, stride;
  if (U.first) {
    if (!unit_of_wave<TPB>(U, n_tiles, wid, unit)) return;
    tile = uint32_t(__builtin_amdgcn_readfirstlane(int(U.tile[unit])));
    chunk = unit - U.first[tile];
    const uint32_t lo = rng[tile].x, hi = rng[tile].y, per = unit_keys(hi - lo);
    b_first = lo + chunk * per;
    b_end = min(hi, b_first + per);
    stride = kWave;
  } else {
    unit = uint32_t(__builtin_amdgcn_readfirstlane(int(xcd_block(blockIdx.x, gridDim.x) * TPB + wid)));
    if (unit >= n_tiles * uint32_t(n_chunks)) return;
    tile = unit / uint32_t(n_chunks);
    chunk = unit - tile * uint32_t(n_chunks);
    b_first = rng[tile].x + chunk * kWave;
    b_end = rng[tile].y;
    stride = kWave * uint32_t(n_chunks);
  }
  b_first = uint32_t(__builtin_amdgcn_readfirstlane(int(b_first)));
  b_end = uint32_t(__builtin_amdgcn_readfirstlane(int(b_end)));
  chunk = uint32_t(__builtin_amdgcn_readfirstlane(int(chunk)));
  const uint32_t v_local = tile / uint32_t(tpv);
  const uint32_t t = tile - v_local * uint32_t(tpv);
  const int ty = int(t) / tiles_x;
  const int tx = int(t) - ty * tiles_x;
  const int lane = threadIdx.x & (kWave - 1);
  // 16-lane group grp owns quadrant grp. Its two 8-lane halves take two pairs
  // of the quadrant's list at a time (entries i and i + 1), each lane a
  // whole column of the quadrant (8 pixels); the halves' sums of the same
  // pixels are added once at the end.
  const int grp = lane >> 4;
  const int half = (lane >> 3) & 1;
  const int col = (grp & 1) * 8 + (lane & 7);
  const int row0 = (grp >> 1) * 8;
  const float px = float(tx * kTS + col) + 0.5f;
  const float py = float(ty * kTS + row0) + 0.5f;
  const float tx0 = float(tx * kTS) + 0.5f, ty0 = float(ty * kTS) + 0.5f;
  if (lane == 0) {
    s_cw[kWave] = make_float4(-1.f, 0.f, -1.f, 0.f);
    s_xy[kWave] = make_float4(-1.0e4f, -1.0e4f, -2.f, 0.f);
  }
  float acc[kFwdRows];
#pragma unroll
  for (int k = 0; k < kFwdRows; ++k) acc[k] = 0.f;
  const uint32_t e = b_end;
  BatchPrefetch<SplatRec> pf;
  pf.start(svals, rec, b_first, stride, e, lane);
  for (uint32_t b = b_first; b < e; b += stride) {
    const uint32_t m = min(uint32_t(kWave), e - b);
    pf.advance(svals, rec, b, stride, e, lane);
    uint32_t mask = 0, imask = 0;
    if (uint32_t(lane) < m) {
      const float4 ra = pf.cur.a;
      const float2 rb = make_float2(pf.cur.b.x, pf.cur.b.y);
      const float4 c = make_float4(ra.z, ra.w, rb.x, rb.y);
      const float2 q = make_float2(ra.x, ra.y);
      const float thr_r = support_thr(thr, log2_tau, c.w);
      s_cw[lane] = c;
      s_xy[lane] = make_float4(q.x, q.y, 2.f * c.z, thr_r);
      mask = no_cull ? 0xFu : quad_mask(c, q.x, q.y, tx0, ty0, thr_r * kCullSlack);
      if (kInterior && !kCount) imask = quad_interior(c, q.x, q.y, tx0, ty0, thr_r * kInteriorSlack) & mask;
    }
    int nq[4], ni[4] = {0, 0, 0, 0};
    if (kInterior && !kCount) {
      build_quad_lists_split(mask, imask, lane, s_list, nq, ni);
    } else {
      int pos[4];
      build_quad_lists(mask, lane, s_list, nq, pos);
    }
    const int n_max = max(max(nq[0], nq[1]), max(nq[2], nq[3]));
    // the lists are padded with the null slot to n_max rounded up to even
    const int n_pad = (n_max + 1) & ~1;
#pragma unroll
    for (int Q = 0; Q < 4; ++Q)
      if (lane >= nq[Q] && lane < n_pad) s_list[Q][lane] = uint8_t(kWave);
    // iterations in which every group's two pairs are interior skip the cutoff test
    const int n_fast = (kInterior && !kCount) ? (min(min(ni[0], ni[1]), min(ni[2], ni[3])) & ~1) : 0;
    wave_lds_sync();
    for (int i = 0; i < n_fast; i += 2) {
      const int j = int(s_list[grp][i + half]);
      const float4 c = s_cw[j];
      const float4 q = s_xy[j];
      const float dx = px - q.x;
      const float dy = py - q.y;
      const float A = c.x * dx * dx;
      const float B = c.y * dx;
      const float arg0 = fmaf(dy, fmaf(c.z, dy, B), A);
      const float E = fmaf(q.z, dy, B);
#pragma unroll
      for (int k = 0; k < kFwdRows; ++k) {
        const float fk = float(k);
        const float arg = (k == 0) ? arg0 : fmaf(fk, fmaf(c.z, fk, E), arg0);
        acc[k] = fmaf(c.w, __builtin_amdgcn_exp2f(arg), acc[k]);
      }
    }
    for (int i = n_fast; i < n_max; i += 2) {
      const int j = int(s_list[grp][i + half]);
      const float4 c = s_cw[j];
      const float4 q = s_xy[j];
      const float dx = px - q.x;
      const float dy = py - q.y;
      const float A = c.x * dx * dx;
      const float B = c.y * dx;
      // exponent down the lane's column, expanded about its first pixel:
      // arg(dy + k) = arg0 + k (2 c.z dy + B) + c.z k^2
      const float arg0 = fmaf(dy, fmaf(c.z, dy, B), A);
      const float E = fmaf(q.z, dy, B);
#pragma unroll
      for (int k = 0; k < kFwdRows; ++k) {
        const float fk = float(k);
        const float arg = (k == 0) ? arg0 : fmaf(fk, fmaf(c.z, fk, E), arg0);
        const float cut = kTau ? q.w : thr;
        if (kCount) {
          acc[k] += (arg >= cut) ? 1.f : 0.f;
        } else {
          const float ex = __builtin_amdgcn_exp2f(arg);
          acc[k] = fmaf(c.w, (arg >= cut) ? ex : 0.f, acc[k]);
        }
      }
    }
    wave_lds_sync();
  }
  const int x = tx * kTS + col;
  if (kCount) {
    // both halves count their own pairs; the wave total is the tile's
    unsigned long long n = 0;
#pragma unroll
    for (int k = 0; k < kFwdRows; ++k) {
      const int y = ty * kTS + row0 + k;
      if (x < W && y < H) n += static_cast<unsigned long long>(acc[k]);
    }
    for (int d = 32; d > 0; d >>= 1) n += __shfl_xor(n, d, 64);
    if (lane == 0 && n) atomicAdd(counter, n);
    return;
  }
  // half 0 adds half 1's sums of the same pixels (lane + 8) and writes
#pragma unroll
  for (int k = 0; k < kFwdRows; ++k) acc[k] += __shfl_down(acc[k], 8, kWave);
  if (half) return;
  if (U.first) {
    // the unit's own 16 x 16 slot; every pixel is written
    float *slot = img + uint64_t(unit) * (kTS * kTS);
#pragma unroll
    for (int k = 0; k < kFwdRows; ++k) slot[(row0 + k) * kTS + col] = acc[k];
    return;
  }
  float *out = img + (uint64_t(chunk) * (n_tiles / uint32_t(tpv)) + v_local) * uint64_t(W) * uint64_t(H);
#pragma unroll
  for (int k = 0; k < kFwdRows; ++k) {
    const int y = ty * kTS + row0 + k;
    if (x < W && y < H) out[uint64_t(y) * W + x] = acc[k];
  }
}

__device__ __forceinline__ float bperm(int src_lane, float v) {
  return __int_as_float(__builtin_amdgcn_ds_bpermute(src_lane << 2, __float_as_int(v)));
}

// Backward over one tile (per-Gaussian formulation). The (quadrant, Gaussian)
// pairs of a batch form one list, quadrant by quadrant; each round the 64
// lanes take the next 64 pairs, so rounds are full whatever the split over
// quadrants. A lane owns one pair and sums over the quadrant's 64 pixels
// (dL/dI read from LDS) the six moments sum g e {1, dx, dy, dx^2, dx dy,
// dy^2}, (dx, dy) = pixel - centre. Pixel coordinates are taken relative to
// the quadrant centre, (cc, rr) in {-3.5, ..., 3.5}: per row the exponent is
// a quadratic in cc with lane coefficients and the moments are accumulated
// against the constants cc, cc^2 (branch-free body), then moved to the
// Gaussian's centre. The lane that loaded a record gathers its up to four
// quadrant partials with wavefront permutes, in quadrant order, and writes
// the pair's six sums to the pair's emission slot: no atomics, and the
// summation order is fixed. 72 registers (7 waves per SIMD): at 64 the
// round loop spilled, and 72 measured 2% faster on 512^2 views.
// kTau: the density-aware support, whose per-record threshold the pixel
// loop reads from LDS; without it the loop compares with the kernel argument.
template <int TPB, bool kTau>
__global__ __launch_bounds__(kWave * TPB) __attribute__((amdgpu_waves_per_eu(7, 7))) void splat_bwd_kernel(
    const uint2 *__restrict__ rng, const ListRecs svals,
    const SplatRec *__restrict__ rec, int tiles_x, int tpv, int W, int H, uint32_t n_tiles, int n_chunks,
    Units U, float thr, float log2_tau, int no_cull, const float *__restrict__ gimg,
    float4 *__restrict__ partials) {
  // per pixel: g = dL/dI and g cc (cc: column relative to the quadrant
  // centre), so the row loop accumulates with three FMAs per pixel
  __shared__ float4 s_g4_all[TPB][2][kTS * kTS / 4];
  __shared__ float4 s_cw_all[TPB][kWave + 1];
  __shared__ float2 s_xy_all[TPB][kWave + 1];
  __shared__ uint8_t s_cat_all[TPB][4 * kWave];
  const int wid = threadIdx.x / kWave;
  float4 *s_g4 = s_g4_all[wid][0];
  float *s_g = reinterpret_cast<float *>(s_g4);
  float4 *s_cw = s_cw_all[wid];
  float2 *s_xy = s_xy_all[wid];
  uint8_t *s_cat = s_cat_all[wid];
  // work unit: a piece of a tile's list (U.first, tiles in row order), or
  // (tile, chunk) where chunk c takes batches c, c + n_chunks, ... (each
  // pair's sums go to its own slot, so units are independent). Everything
  // about the unit is the same across the wave (kept in scalar registers).
  uint32_t unit, rt, v_local, b_first, b_end, stride;
  int tx, ty;
  if (U.first) {
    if (!unit_of_wave<TPB>(U, n_tiles, wid, unit)) return;
    rt = uint32_t(__builtin_amdgcn_readfirstlane(int(U.tile[unit])));
    const uint32_t chunk = unit - U.first[rt];
    v_local = rt / uint32_t(tpv);
    const uint32_t t = rt - v_local * uint32_t(tpv);
    ty = int(t) / tiles_x;
    tx = int(t) - ty * tiles_x;
    const uint32_t lo = rng[rt].x, hi = rng[rt].y, per = unit_keys(hi - lo);
    b_first = lo + chunk * per;
    b_end = min(hi, b_first + per);
    stride = kWave;
    if (b_first >= b_end) return;  // an empty tile: nothing to write
  } else {
    unit = uint32_t(__builtin_amdgcn_readfirstlane(int(xcd_block(blockIdx.x, gridDim.x) * TPB + wid)));
    if (unit >= n_tiles * uint32_t(n_chunks)) return;
    const uint32_t tile = unit / uint32_t(n_chunks);
    const uint32_t chunk = unit - tile * uint32_t(n_chunks);
    v_local = tile / uint32_t(tpv);
    const uint32_t t = tile - v_local * uint32_t(tpv);
    tile_of(t, tiles_x, tpv / tiles_x, tx, ty);
    rt = v_local * uint32_t(tpv) + uint32_t(ty * tiles_x + tx);
    b_first = rng[rt].x + chunk * kWave;
    b_end = rng[rt].y;
    stride = kWave * uint32_t(n_chunks);
  }
  b_first = uint32_t(__builtin_amdgcn_readfirstlane(int(b_first)));
  b_end = uint32_t(__builtin_amdgcn_readfirstlane(int(b_end)));
  const int lane = threadIdx.x & (kWave - 1);
  const float *gv = gimg + uint64_t(v_local) * uint64_t(W) * uint64_t(H);
  for (int p = lane; p < kTS * kTS; p += kWave) {
    const int x = tx * kTS + (p & (kTS - 1));
    const int y = ty * kTS + (p >> 4);
    const float g = (x < W && y < H) ? gv[uint64_t(y) * W + x] : 0.f;
    const float cc = float(p & 7) - 3.5f;
    s_g[p] = g;
    s_g[kTS * kTS + p] = g * cc;
  }
  if (lane == 0) set_null_record(s_cw, s_xy);
  wave_lds_sync();
  const float tx0 = float(tx * kTS) + 0.5f, ty0 = float(ty * kTS) + 0.5f;
  const uint64_t lt = (lane == 0) ? 0ull : (~0ull >> (64 - lane));
  const uint32_t e = b_end;
  for (uint32_t b = b_first; b < e; b += stride) {
    const uint32_t m = min(uint32_t(kWave), e - b);
    uint32_t mask = 0, slot = 0;
    if (uint32_t(lane) < m) {
      const uint32_t r = svals[b + lane];
      const float4 ra = rec[r].a, rb = rec[r].b;
      const float4 c = make_float4(ra.z, ra.w, rb.x, rb.y);
      const float2 q = make_float2(ra.x, ra.y);
      slot = __float_as_uint(rb.z) + uint32_t(ty) * __float_as_uint(rb.w) + uint32_t(tx);
      // the pixel loop needs no weight: the record's support threshold takes its place
      const float thr_r = support_thr(thr, log2_tau, c.w);
      s_cw[lane] = make_float4(c.x, c.y, c.z, thr_r);
      s_xy[lane] = q;
      mask = no_cull ? 0xFu : quad_mask(c, q.x, q.y, tx0, ty0, thr_r * kCullSlack);
    }
    // one list of (quadrant << 6 | batch slot) entries, quadrant-major; gpk
    // holds this lane's record's position in it for each quadrant (8 bits each)
    int n_pairs = 0;
    uint32_t gpk = 0;
#pragma unroll
    for (int Q = 0; Q < 4; ++Q) {
      const bool bit = (mask >> Q) & 1u;
      const uint64_t bal = __ballot(bit);
      const int gp = n_pairs + __popcll(bal & lt);
      if (bit) s_cat[gp] = uint8_t((Q << 6) | lane);
      gpk |= uint32_t(gp & 255) << (8 * Q);
      n_pairs += __popcll(bal);
    }
    wave_lds_sync();
    float tot[6] = {0.f, 0.f, 0.f, 0.f, 0.f, 0.f};
    for (int base = 0; base < n_pairs;) {
      // a round with at most 32 pairs left spreads each pair's 8 rows over
      // 2, 4 or 8 lanes (lane = part * P + pair); the parts are summed in a
      // fixed tree below, so the result stays deterministic
      const int rem = n_pairs - base;
      const int lg = rem > 32 ? 0 : rem > 16 ? 1 : rem > 8 ? 2 : 3;
      const int P = kWave >> lg;
      const int nrows = 8 >> lg;
      const int row0 = (lane >> (6 - lg)) * nrows;
      const float rr0 = float(row0) - 3.5f;
      const int idx = base + (lane & (P - 1));
      int Q = 0, j = kWave;
      if (idx < n_pairs) {
        const int ent = s_cat[idx];
        Q = ent >> 6;
        j = ent & 63;
      }
      // centre of the pair's quadrant and its first float4 of dL/dI
      const float ox = float(tx * kTS + (Q & 1) * 8) + 4.f;
      const float oy = float(ty * kTS + (Q >> 1) * 8) + 4.f;
      const float4 *g4q = s_g4 + ((Q >> 1) * 8 + row0) * (kTS / 4) + (Q & 1) * 2;
      const float4 c = s_cw[j];
      const float2 q = s_xy[j];
      // Gaussian centre relative to the quadrant centre; arg = c.x dx^2 + c.y dx dy + c.z dy^2
      const float qx = q.x - ox, qy = q.y - oy;
      const float m2aqx = -2.f * c.x * qx;
      const float aqx2 = c.x * qx * qx;
      const float mbqx = -c.y * qx;
      // per column: A = sum over rows of g e; per row: sum over columns of
      // g e and of g e cc, folded into the row moments
      float A[8] = {0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f};
      float Sr = 0.f, Scr = 0.f, Srr = 0.f;
#pragma unroll 1
      for (int row = 0; row < nrows; ++row) {
        const float rr = rr0 + float(row);
        const float dy = rr - qy;
        const float brow = fmaf(c.y, dy, m2aqx);
        const float drow = fmaf(dy, fmaf(c.z, dy, mbqx), aqx2);
        float R0 = 0.f, R1 = 0.f;
#pragma unroll
        for (int qd = 0; qd < 2; ++qd) {
          const float4 g0 = g4q[row * (kTS / 4) + qd];
          const float4 g1 = g4q[kTS * kTS / 4 + row * (kTS / 4) + qd];
          const float G0[4] = {g0.x, g0.y, g0.z, g0.w};
          const float G1[4] = {g1.x, g1.y, g1.z, g1.w};
#pragma unroll
          for (int u = 0; u < 4; ++u) {
            const float cc = float(qd * 4 + u) - 3.5f;
            const float arg = fmaf(cc, fmaf(c.x, cc, brow), drow);
            const float ex = (arg >= (kTau ? c.w : thr)) ? __builtin_amdgcn_exp2f(arg) : 0.f;
            A[qd * 4 + u] = fmaf(G0[u], ex, A[qd * 4 + u]);
            R0 = fmaf(G0[u], ex, R0);
            R1 = fmaf(G1[u], ex, R1);
          }
        }
        Sr = fmaf(R0, rr, Sr);
        Scr = fmaf(R1, rr, Scr);
        Srr = fmaf(R0, rr * rr, Srr);
      }
      float S0 = 0.f, Sc = 0.f, Scc = 0.f;
#pragma unroll
      for (int col = 0; col < 8; ++col) {
        const float cc = float(col) - 3.5f;
        S0 += A[col];
        Sc = fmaf(A[col], cc, Sc);
        Scc = fmaf(A[col], cc * cc, Scc);
      }
      // moments about the Gaussian centre: dx = cc - qx, dy = rr - qy
      float M[6];
      M[0] = S0;
      M[1] = fmaf(-qx, S0, Sc);
      M[2] = fmaf(-qy, S0, Sr);
      M[3] = fmaf(qx * qx, S0, fmaf(-2.f * qx, Sc, Scc));
      M[4] = fmaf(qx * qy, S0, fmaf(-qy, Sc, fmaf(-qx, Sr, Scr)));
      M[5] = fmaf(qy * qy, S0, fmaf(-2.f * qy, Sr, Srr));
      // parts summed pairwise (halves, then quarters, ...) into lanes < P
      for (int off = kWave / 2; off >= P; off >>= 1) {
        const int src = (lane + off) & (kWave - 1);
#pragma unroll
        for (int k = 0; k < 6; ++k) M[k] += bperm(src, M[k]);
      }
      // the loading lane of each record collects its quadrants' partials from
      // this round's lanes (quadrants with no pair in the round are skipped)
#pragma unroll
      for (int QQ = 0; QQ < 4; ++QQ) {
        const int rel = int((gpk >> (8 * QQ)) & 255u) - base;
        const bool mine = ((mask >> QQ) & 1u) && rel >= 0 && rel < P;
        if (__ballot(mine) == 0ull) continue;
        const int src = mine ? rel : 0;
#pragma unroll
        for (int k = 0; k < 6; ++k) {
          const float v = bperm(src, M[k]);
          tot[k] += mine ? v : 0.f;
        }
      }
      base += P;
    }
    if (uint32_t(lane) < m) {
      partials[2 * uint64_t(slot) + 0] = make_float4(tot[0], tot[1], tot[2], tot[3]);
      partials[2 * uint64_t(slot) + 1] = make_float4(tot[4], tot[5], 0.f, 0.f);
    }
    wave_lds_sync();
  }
}

// Ablation only (FGS_ABLATE_PER_PIXEL_BWD): the pixel-parallel backward of
// the original splatting. One wave per tile, each lane a column of 4 pixels;
// for every listed Gaussian each lane forms its pixels' six moment terms,
// the wave sums them (butterfly) and one lane adds them to the record's
// accumulator acc6[r][6] with float atomics. Not deterministic.
__global__ __launch_bounds__(kWave) void splat_bwd_pixel_kernel(
    const uint2 *__restrict__ rng, const ListRecs svals, const SplatRec *__restrict__ rec,
    int tiles_x, int tpv, int W, int H, uint32_t n_tiles, float thr, const float *__restrict__ gimg,
    float *__restrict__ acc6) {
  __shared__ float4 s_cw[kWave];
  __shared__ float2 s_xy[kWave];
  __shared__ uint32_t s_r[kWave];
  const uint32_t tile = blockIdx.x;
  if (tile >= n_tiles) return;
  const uint32_t v_local = tile / uint32_t(tpv);
  const uint32_t t = tile - v_local * uint32_t(tpv);
  const int ty = int(t) / tiles_x;
  const int tx = int(t) - ty * tiles_x;
  const int lane = threadIdx.x;
  const int col = lane & 15, row0 = (lane >> 4) * kRows;
  const float px = float(tx * kTS + col) + 0.5f;
  const float *gv = gimg + uint64_t(v_local) * uint64_t(W) * uint64_t(H);
  float gpx[kRows];
#pragma unroll
  for (int k = 0; k < kRows; ++k) {
    const int x = tx * kTS + col, y = ty * kTS + row0 + k;
    gpx[k] = (x < W && y < H) ? gv[uint64_t(y) * W + x] : 0.f;
  }
  const uint32_t b0 = rng[tile].x, e = rng[tile].y;
  for (uint32_t b = b0; b < e; b += kWave) {
    const uint32_t m = min(uint32_t(kWave), e - b);
    if (uint32_t(lane) < m) {
      const uint32_t r = svals[b + lane];
      const float4 ra = rec[r].a, rb = rec[r].b;
      s_cw[lane] = make_float4(ra.z, ra.w, rb.x, rb.y);
      s_xy[lane] = make_float2(ra.x, ra.y);
      s_r[lane] = r;
    }
    wave_lds_sync();
    for (uint32_t j = 0; j < m; ++j) {
      const float4 c = s_cw[j];
      const float2 q = s_xy[j];
      const float dx = px - q.x;
      float mo[6] = {0.f, 0.f, 0.f, 0.f, 0.f, 0.f};
#pragma unroll
      for (int k = 0; k < kRows; ++k) {
        const float dy = float(ty * kTS + row0 + k) + 0.5f - q.y;
        const float arg = fmaf(dx, fmaf(c.x, dx, c.y * dy), c.z * dy * dy);
        const float ge = ((arg >= thr) ? gpx[k] : 0.f) * __builtin_amdgcn_exp2f(arg);
        mo[0] += ge;
        mo[1] = fmaf(ge, dx, mo[1]);
        mo[2] = fmaf(ge, dy, mo[2]);
        mo[3] = fmaf(ge * dx, dx, mo[3]);
        mo[4] = fmaf(ge * dx, dy, mo[4]);
        mo[5] = fmaf(ge * dy, dy, mo[5]);
      }
#pragma unroll
      for (int d = 32; d > 0; d >>= 1)
#pragma unroll
        for (int i = 0; i < 6; ++i) mo[i] += __shfl_xor(mo[i], d, 64);
      if (lane == 0) {
        float *a = acc6 + 6 * uint64_t(s_r[j]);
#pragma unroll
        for (int i = 0; i < 6; ++i) unsafeAtomicAdd(a + i, mo[i]);
      }
    }
    wave_lds_sync();
  }
}

__global__ __launch_bounds__(256) void fill_zero_kernel(float *__restrict__ p, uint64_t n) {
  const uint64_t i = uint64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (i < n) p[i] = 0.f;
}

// Per record: reduce its contiguous partial slots, then the chain rule to
// the 11 parameters. A block takes 256 consecutive records of one view. The
// slots are read by groups of kGradLanes lanes, one record per group at a
// time, each lane taking every kGradLanes-th slot (consecutive lanes read
// consecutive 32-byte slots), then summed across the group in a fixed
// butterfly order; one thread per record then applies the chain rule.
constexpr int kGradLanes = 8;
constexpr int kGradUnroll = 4;

// A record's 11 gradient components: to grad_rec[c][r] (summed over the
// views afterwards), or, for a one-view call (kDirect), straight into the
// output arrays (added to them with accumulate), as view_sum_kernel would.
struct GradSink {
  float *__restrict__ grad_rec;
  uint64_t R;
  fgs_gaussian_grads out;
  int accumulate;
  template <bool kDirect>
  __device__ __forceinline__ void put(int c, uint64_t r, int64_t i, int64_t n, float val) const {
    if constexpr (!kDirect) {
      grad_rec[uint64_t(c) * R + r] = val;
    } else {
      float *d = c < 3 ? out.mean + c * n : (c < 6 ? out.log_scale + (c - 3) * n
                                                   : (c < 10 ? out.quat + (c - 6) * n : out.density));
      d[i] = accumulate ? d[i] + val : val;
    }
  }
};

template <int RPB, bool kDirect>
__global__ __launch_bounds__(256) void record_grad_kernel(fgs_gaussians g, GeomDev G,
                                                          const uint32_t *__restrict__ offset,
                                                          const float4 *__restrict__ partials,
                                                          const float *__restrict__ acc6, uint64_t R,
                                                          const uint32_t *__restrict__ kdev, GradSink sink) {
  __shared__ float s_sum[RPB][7];
  __shared__ uint32_t s_off[RPB + 1];
  // kdev[1]: the lists overflowed their capacity and hold nothing
  const bool none = kdev[1] != 0u;
  const int t = threadIdx.x;
  const int64_t i0 = int64_t(blockIdx.x) * RPB;
  const int v_local = blockIdx.y;
  const uint64_t rbase = uint64_t(v_local) * uint64_t(g.n);
  // the block's RPB + 1 offsets in one coalesced read (offset has R + 1 entries)
  for (int j = t; j <= RPB; j += 256)
    if (i0 + j <= g.n) s_off[j] = offset[rbase + uint64_t(i0 + j)];
  __syncthreads();
  const int li = t % kGradLanes;
  for (int idx = t / kGradLanes; idx < RPB && !acc6; idx += 256 / kGradLanes) {
    if (i0 + idx >= g.n || none) break;
    const uint32_t o = s_off[idx], end = s_off[idx + 1];
    if (o == end) continue;  // the whole lane group agrees: no pairs, nothing to sum
    float acc[6] = {0.f, 0.f, 0.f, 0.f, 0.f, 0.f};
    {
      // kGradUnroll slots' loads in flight at a time; summed in slot order
      for (uint32_t p = o + li; p < end; p += kGradUnroll * kGradLanes) {
        float4 a[kGradUnroll];
        float2 b[kGradUnroll];
#pragma unroll
        for (int u = 0; u < kGradUnroll; ++u) {
          const uint32_t pp = p + uint32_t(u * kGradLanes);
          a[u] = pp < end ? partials[2 * uint64_t(pp) + 0] : make_float4(0.f, 0.f, 0.f, 0.f);
          b[u] = pp < end ? *reinterpret_cast<const float2 *>(&partials[2 * uint64_t(pp) + 1]) : make_float2(0.f, 0.f);
        }
#pragma unroll
        for (int u = 0; u < kGradUnroll; ++u) {
          if (p + uint32_t(u * kGradLanes) >= end) break;
          acc[0] += a[u].x; acc[1] += a[u].y; acc[2] += a[u].z;
          acc[3] += a[u].w; acc[4] += b[u].x; acc[5] += b[u].y;
        }
      }
    }
#pragma unroll
    for (int d = 1; d < kGradLanes; d <<= 1)
#pragma unroll
      for (int c = 0; c < 6; ++c) acc[c] += __shfl_xor(acc[c], d, kGradLanes);
    if (li == 0)
#pragma unroll
      for (int c = 0; c < 6; ++c) s_sum[idx][c] = acc[c];
  }
  __syncthreads();
  const int64_t i = i0 + t;
  if (t >= RPB || i >= g.n) return;
  const uint64_t r = rbase + uint64_t(i);
  float out[11];
  if (none || s_off[t] == s_off[t + 1]) {
#pragma unroll
    for (int c = 0; c < 11; ++c) sink.put<kDirect>(c, r, i, g.n, 0.f);
    return;
  }
  float sums[6];
#pragma unroll
  for (int c = 0; c < 6; ++c) sums[c] = acc6 ? acc6[6 * r + c] : s_sum[t][c];
  GaussParams P;
  load_gauss(g, i, P);
  ViewFrame F;
  make_frame(G, G.view_begin + v_local, F);
  Splat S;
  splat_forward(P, F, G, S);
  if (!S.ok) {
#pragma unroll
    for (int c = 0; c < 11; ++c) sink.put<kDirect>(c, r, i, g.n, 0.f);
    return;
  }
  // moments are relative to the pixel coordinate frame: the sums use
  // (pixel - centre); the kernel's pre-scaled conic is undone here
  splat_backward(P, F, G, S, sums, out);
#pragma unroll
  for (int c = 0; c < 11; ++c) sink.put<kDirect>(c, r, i, g.n, out[c]);
}

__global__ __launch_bounds__(256) void view_sum_kernel(int64_t n, int views,
                                                       const float *__restrict__ grad_rec,
                                                       fgs_gaussian_grads out, int accumulate) {
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
  if (accumulate) {
    acc[0] += out.mean[i]; acc[1] += out.mean[n + i]; acc[2] += out.mean[2 * n + i];
    acc[3] += out.log_scale[i]; acc[4] += out.log_scale[n + i]; acc[5] += out.log_scale[2 * n + i];
    acc[6] += out.quat[i]; acc[7] += out.quat[n + i]; acc[8] += out.quat[2 * n + i]; acc[9] += out.quat[3 * n + i];
    acc[10] += out.density[i];
  }
  out.mean[i] = acc[0]; out.mean[n + i] = acc[1]; out.mean[2 * n + i] = acc[2];
  out.log_scale[i] = acc[3]; out.log_scale[n + i] = acc[4]; out.log_scale[2 * n + i] = acc[5];
  out.quat[i] = acc[6]; out.quat[n + i] = acc[7]; out.quat[2 * n + i] = acc[8]; out.quat[3 * n + i] = acc[9];
  out.density[i] = acc[10];
}

// ---------------------------------------------------------------- ray-exact pixel kernels
//
// Same tiling, quadrant culling (against the support ellipse of the model)
// and lists as the splat kernels; per pixel the exact line integral of the
// record's Gaussian (exact_math.h) replaces the splat:
//   A = a0 + 2 l.delta + delta^T K delta, C = delta^T C delta,
//   contribution w A^-1/2 exp2(escale C / A) where escale C / A >= thr,
// and the pixel's |d| multiplies the sum (forward) or dL/dI (backward).

// Quadrant mask of a ray-exact record (all four quadrants if the support
// ellipse comes out degenerate in FP32: the per-pixel test then decides).
__device__ __forceinline__ uint32_t exact_quad_mask(const float4 &ra, const float4 &rb, const float4 &rc, float k2,
                                                    float tx0, float ty0, float thr_cull) {
  float dcx, dcy, hx, hy, cs00, cs01, cs11;
  const float t2sq = -2.f * kLn2 * rc.w;
  if (!exact_silhouette(ra.z, ra.w, rb.x, rb.y, rb.z, rb.w, rc.x, rc.y, rc.z, t2sq, k2, dcx, dcy, hx, hy, cs00,
                        cs01, cs11))
    return 0xFu;
  const float k = -0.5f * kLog2e;
  const float4 c = make_float4(k * cs00, 2.f * k * cs01, k * cs11, 0.f);
  return quad_mask(c, ra.x + dcx, ra.y + dcy, tx0, ty0, thr_cull);
}

// |d| of the ray through pixel coordinate (x, y): the arc length per unit depth.
__device__ __forceinline__ float ray_length(float x, float y, float fu, float fv, float cu, float cv) {
  const float s = (x - cu) / fu, r = (y - cv) / fv;
  return sqrtf(fmaf(s, s, fmaf(r, r, 1.f)));
}

// A record that contributes nothing: zero weight, exponent far below thr.
__device__ __forceinline__ void set_null_exact(float4 *s_a, float4 *s_b, float4 *s_c) {
  s_a[kWave] = make_float4(-1.0e4f, -1.0e4f, 0.f, 0.f);
  s_b[kWave] = make_float4(0.f, 0.f, 0.f, 1.f);
  s_c[kWave] = make_float4(1.f, 0.f, 1.f, -1.f);
}

struct ExactCam {
  float fu, fv, cu, cv, k2;
};

template <bool kCount, int TPB>
__global__ __launch_bounds__(kWave * TPB) void splat_fwd_exact_kernel(
    const uint2 *__restrict__ rng, const ListRecs svals, const ExactRec *__restrict__ rec,
    int tiles_x, int tpv, int W, int H, uint32_t n_tiles, int n_chunks, float thr, float thr_cull, ExactCam cam,
    float *__restrict__ img, unsigned long long *__restrict__ counter) {
  __shared__ float4 s_a_all[TPB][kWave + 1];
  __shared__ float4 s_b_all[TPB][kWave + 1];
  __shared__ float4 s_c_all[TPB][kWave + 1];
  __shared__ float s_w_all[TPB][kWave + 1];
  __shared__ uint8_t s_list_all[TPB][4][kWave];
  const int wid = threadIdx.x / kWave;
  float4 *s_a = s_a_all[wid];
  float4 *s_b = s_b_all[wid];
  float4 *s_c = s_c_all[wid];
  float *s_w = s_w_all[wid];
  uint8_t(*s_list)[kWave] = s_list_all[wid];
  const uint32_t unit = xcd_block(blockIdx.x, gridDim.x) * TPB + wid;
  if (unit >= n_tiles * uint32_t(n_chunks)) return;
  const uint32_t tile = unit / uint32_t(n_chunks);
  const uint32_t chunk = unit - tile * uint32_t(n_chunks);
  const uint32_t v_local = tile / uint32_t(tpv);
  const uint32_t t = tile - v_local * uint32_t(tpv);
  const int ty = int(t) / tiles_x;
  const int tx = int(t) - ty * tiles_x;
  const uint32_t rt = tile;
  const int lane = threadIdx.x & (kWave - 1);
  const int grp = lane >> 4;
  const int sub = lane & 15;
  const int col = (grp & 1) * 8 + (sub & 7);
  const int row0 = (grp >> 1) * 8 + (sub >> 3) * kRows;
  const float px = float(tx * kTS + col) + 0.5f;
  const float py = float(ty * kTS + row0) + 0.5f;
  const float tx0 = float(tx * kTS) + 0.5f, ty0 = float(ty * kTS) + 0.5f;
  if (lane == 0) {
    set_null_exact(s_a, s_b, s_c);
    s_w[kWave] = 0.f;
  }
  float acc[kRows];
#pragma unroll
  for (int k = 0; k < kRows; ++k) acc[k] = 0.f;
  const uint32_t b0 = rng[rt].x, e = rng[rt].y;
  for (uint32_t b = b0 + chunk * kWave; b < e; b += kWave * uint32_t(n_chunks)) {
    const uint32_t m = min(uint32_t(kWave), e - b);
    uint32_t mask = 0;
    if (uint32_t(lane) < m) {
      const uint32_t r = svals[b + lane];
      const float4 ra = rec[r].a, rb = rec[r].b, rc = rec[r].c;
      s_a[lane] = ra;
      s_b[lane] = rb;
      s_c[lane] = rc;
      s_w[lane] = rec[r].d.x;
      mask = exact_quad_mask(ra, rb, rc, cam.k2, tx0, ty0, thr_cull);
    }
    int nq[4], pos[4];
    build_quad_lists(mask, lane, s_list, nq, pos);
    const int n_max = max(max(nq[0], nq[1]), max(nq[2], nq[3]));
#pragma unroll
    for (int Q = 0; Q < 4; ++Q)
      if (lane >= nq[Q] && lane < n_max) s_list[Q][lane] = uint8_t(kWave);
    wave_lds_sync();
    for (int i = 0; i < n_max; ++i) {
      const int j = int(s_list[grp][i]);
      const float4 ra = s_a[j], rb = s_b[j], rc = s_c[j];
      const float w = s_w[j];
      const float dx = px - ra.x;
      const float dy0 = py - ra.y;
      const float Kx = ra.z * dx * dx, K1 = 2.f * ra.w * dx;
      const float Cx = rc.x * dx * dx, C1 = 2.f * rc.y * dx;
      const float Lx = rb.y * dx;
#pragma unroll
      for (int k = 0; k < kRows; ++k) {
        const float dy = dy0 + float(k);
        const float K = fmaf(dy, fmaf(rb.x, dy, K1), Kx);
        const float C = fmaf(dy, fmaf(rc.z, dy, C1), Cx);
        const float L = fmaf(rb.z, dy, Lx);
        const float A = fmaf(2.f, L, rb.w + K);
        const float ri = __builtin_amdgcn_rsqf(A);
        const float arg = rc.w * C * (ri * ri);
        if (kCount) {
          acc[k] += (arg >= thr) ? 1.f : 0.f;
        } else {
          const float ex = __builtin_amdgcn_exp2f(arg);
          acc[k] = fmaf(w * ri, (arg >= thr) ? ex : 0.f, acc[k]);
        }
      }
    }
    wave_lds_sync();
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
  float *out = img + (uint64_t(chunk) * (n_tiles / uint32_t(tpv)) + v_local) * uint64_t(W) * uint64_t(H);
#pragma unroll
  for (int k = 0; k < kRows; ++k) {
    const int y = ty * kTS + row0 + k;
    if (x < W && y < H) out[uint64_t(y) * W + x] = acc[k] * ray_length(px, py + float(k), cam.fu, cam.fv, cam.cu, cam.cv);
  }
}

// Number of per-pair sums of the ray-exact backward (exact_backward's s[]);
// a pair's slot holds them in 16 floats (64 bytes).
constexpr int kExactSums = 13;

// Backward of the ray-exact model over one tile, organised as the splat
// backward: one lane per (quadrant, Gaussian) pair sums over the quadrant's
// 64 pixels, coordinates relative to the quadrant centre; per row the sums
// against the column constants cc, cc^2 are folded with the row constants,
// then moved to the Gaussian's centre. With p = g |d| A^-1/2 exp(phi) the
// sums are those exact_backward takes: sum p, sum p C / A, and the moments
// of alpha = -(p / A)(1/2 + phi) and beta = p / A.
template <int TPB>
__global__ __launch_bounds__(kWave * TPB) void splat_bwd_exact_kernel(
    const uint2 *__restrict__ rng, const ListRecs svals, const ExactRec *__restrict__ rec,
    int tiles_x, int tpv, int W, int H, uint32_t n_tiles, int n_chunks, float thr, float thr_cull, ExactCam cam,
    const float *__restrict__ gimg, float4 *__restrict__ partials) {
  __shared__ float4 s_g4_all[TPB][kTS * kTS / 4];
  __shared__ float4 s_a_all[TPB][kWave + 1];
  __shared__ float4 s_b_all[TPB][kWave + 1];
  __shared__ float4 s_c_all[TPB][kWave + 1];
  __shared__ uint8_t s_cat_all[TPB][4 * kWave];
  const int wid = threadIdx.x / kWave;
  float4 *s_g4 = s_g4_all[wid];
  float *s_g = reinterpret_cast<float *>(s_g4);
  float4 *s_a = s_a_all[wid];
  float4 *s_b = s_b_all[wid];
  float4 *s_c = s_c_all[wid];
  uint8_t *s_cat = s_cat_all[wid];
  const uint32_t unit = xcd_block(blockIdx.x, gridDim.x) * TPB + wid;
  if (unit >= n_tiles * uint32_t(n_chunks)) return;
  const uint32_t tile = unit / uint32_t(n_chunks);
  const uint32_t chunk = unit - tile * uint32_t(n_chunks);
  const uint32_t v_local = tile / uint32_t(tpv);
  const uint32_t t = tile - v_local * uint32_t(tpv);
  int tx, ty;
  tile_of(t, tiles_x, tpv / tiles_x, tx, ty);
  const uint32_t rt = v_local * uint32_t(tpv) + uint32_t(ty * tiles_x + tx);
  const int lane = threadIdx.x & (kWave - 1);
  const float *gv = gimg + uint64_t(v_local) * uint64_t(W) * uint64_t(H);
  for (int p = lane; p < kTS * kTS; p += kWave) {
    const int x = tx * kTS + (p & (kTS - 1));
    const int y = ty * kTS + (p >> 4);
    s_g[p] = (x < W && y < H)
                 ? gv[uint64_t(y) * W + x] * ray_length(float(x) + 0.5f, float(y) + 0.5f, cam.fu, cam.fv, cam.cu, cam.cv)
                 : 0.f;
  }
  if (lane == 0) set_null_exact(s_a, s_b, s_c);
  wave_lds_sync();
  const float tx0 = float(tx * kTS) + 0.5f, ty0 = float(ty * kTS) + 0.5f;
  const uint64_t lt = (lane == 0) ? 0ull : (~0ull >> (64 - lane));
  const uint32_t b0 = rng[rt].x, e = rng[rt].y;
  for (uint32_t b = b0 + chunk * kWave; b < e; b += kWave * uint32_t(n_chunks)) {
    const uint32_t m = min(uint32_t(kWave), e - b);
    uint32_t mask = 0, slot = 0;
    if (uint32_t(lane) < m) {
      const uint32_t r = svals[b + lane];
      const float4 ra = rec[r].a, rb = rec[r].b, rc = rec[r].c, rd = rec[r].d;
      slot = __float_as_uint(rd.y) + uint32_t(ty) * __float_as_uint(rd.z) + uint32_t(tx);
      s_a[lane] = ra;
      s_b[lane] = rb;
      s_c[lane] = rc;
      mask = exact_quad_mask(ra, rb, rc, cam.k2, tx0, ty0, thr_cull);
    }
    int n_pairs = 0;
    uint32_t gpk = 0;
#pragma unroll
    for (int Q = 0; Q < 4; ++Q) {
      const bool bit = (mask >> Q) & 1u;
      const uint64_t bal = __ballot(bit);
      const int gp = n_pairs + __popcll(bal & lt);
      if (bit) s_cat[gp] = uint8_t((Q << 6) | lane);
      gpk |= uint32_t(gp & 255) << (8 * Q);
      n_pairs += __popcll(bal);
    }
    wave_lds_sync();
    float tot[kExactSums];
#pragma unroll
    for (int k = 0; k < kExactSums; ++k) tot[k] = 0.f;
    for (int base = 0; base < n_pairs;) {
      // the last partial round spreads each pair's rows over 2, 4 or 8 lanes,
      // as in the splat backward
      const int rem = n_pairs - base;
      const int lg = rem > 32 ? 0 : rem > 16 ? 1 : rem > 8 ? 2 : 3;
      const int P = kWave >> lg;
      const int nrows = 8 >> lg;
      const int row0 = (lane >> (6 - lg)) * nrows;
      const float rr0 = float(row0) - 3.5f;
      const int idx = base + (lane & (P - 1));
      int Q = 0, j = kWave;
      if (idx < n_pairs) {
        const int ent = s_cat[idx];
        Q = ent >> 6;
        j = ent & 63;
      }
      const float ox = float(tx * kTS + (Q & 1) * 8) + 4.f;
      const float oy = float(ty * kTS + (Q >> 1) * 8) + 4.f;
      const float4 *g4q = s_g4 + ((Q >> 1) * 8 + row0) * (kTS / 4) + (Q & 1) * 2;
      const float4 ra = s_a[j], rb = s_b[j], rc = s_c[j];
      const float qx = ra.x - ox, qy = ra.y - oy;
      float Sw = 0.f, Se = 0.f;
      float a0 = 0.f, ac = 0.f, acc2 = 0.f, ar = 0.f, acr = 0.f, arr = 0.f;
      float b0s = 0.f, bc = 0.f, bcc = 0.f, br = 0.f, bcr = 0.f, brr = 0.f;
#pragma unroll 1
      for (int row = 0; row < nrows; ++row) {
        const float rr = rr0 + float(row);
        const float dy = rr - qy;
        const float Krow1 = 2.f * ra.w * dy, Krow0 = rb.x * dy * dy;
        const float Crow1 = 2.f * rc.y * dy, Crow0 = rc.z * dy * dy;
        const float Lrow = rb.z * dy;
        float Ra0 = 0.f, Ra1 = 0.f, Ra2 = 0.f, Rb0 = 0.f, Rb1 = 0.f, Rb2 = 0.f;
#pragma unroll
        for (int qd = 0; qd < 2; ++qd) {
          const float4 gq = g4q[row * (kTS / 4) + qd];
          const float gcol[4] = {gq.x, gq.y, gq.z, gq.w};
#pragma unroll
          for (int u = 0; u < 4; ++u) {
            const float cc = float(qd * 4 + u) - 3.5f;
            const float dx = cc - qx;
            const float K = fmaf(dx, fmaf(ra.z, dx, Krow1), Krow0);
            const float C = fmaf(dx, fmaf(rc.x, dx, Crow1), Crow0);
            const float L = fmaf(rb.y, dx, Lrow);
            const float A = fmaf(2.f, L, rb.w + K);
            const float ri = __builtin_amdgcn_rsqf(A);
            const float ia = ri * ri;
            const float arg = rc.w * C * ia;
            const float ex = __builtin_amdgcn_exp2f(arg);
            const float p = ((arg >= thr) ? gcol[u] : 0.f) * ri * ex;
            const float be = p * ia;
            const float al = -be * fmaf(arg, kLn2, 0.5f);
            Sw += p;
            Se = fmaf(be, C, Se);
            Ra0 += al;
            Ra1 = fmaf(al, cc, Ra1);
            Ra2 = fmaf(al, cc * cc, Ra2);
            Rb0 += be;
            Rb1 = fmaf(be, cc, Rb1);
            Rb2 = fmaf(be, cc * cc, Rb2);
          }
        }
        a0 += Ra0; ac += Ra1; acc2 += Ra2;
        ar = fmaf(Ra0, rr, ar); acr = fmaf(Ra1, rr, acr); arr = fmaf(Ra0, rr * rr, arr);
        b0s += Rb0; bc += Rb1; bcc += Rb2;
        br = fmaf(Rb0, rr, br); bcr = fmaf(Rb1, rr, bcr); brr = fmaf(Rb0, rr * rr, brr);
      }
      // moments about the Gaussian's centre: dx = cc - qx, dy = rr - qy
      float M[kExactSums];
      M[0] = Sw;
      M[1] = Se;
      M[2] = a0;
      M[3] = fmaf(-qx, a0, ac);
      M[4] = fmaf(-qy, a0, ar);
      M[5] = fmaf(qx * qx, a0, fmaf(-2.f * qx, ac, acc2));
      M[6] = fmaf(qx * qy, a0, fmaf(-qy, ac, fmaf(-qx, ar, acr)));
      M[7] = fmaf(qy * qy, a0, fmaf(-2.f * qy, ar, arr));
      M[8] = fmaf(-qx, b0s, bc);
      M[9] = fmaf(-qy, b0s, br);
      M[10] = fmaf(qx * qx, b0s, fmaf(-2.f * qx, bc, bcc));
      M[11] = fmaf(qx * qy, b0s, fmaf(-qy, bc, fmaf(-qx, br, bcr)));
      M[12] = fmaf(qy * qy, b0s, fmaf(-2.f * qy, br, brr));
      for (int off = kWave / 2; off >= P; off >>= 1) {
        const int src = (lane + off) & (kWave - 1);
#pragma unroll
        for (int k = 0; k < kExactSums; ++k) M[k] += bperm(src, M[k]);
      }
#pragma unroll
      for (int QQ = 0; QQ < 4; ++QQ) {
        const int rel = int((gpk >> (8 * QQ)) & 255u) - base;
        const bool mine = ((mask >> QQ) & 1u) && rel >= 0 && rel < P;
        if (__ballot(mine) == 0ull) continue;
        const int src = mine ? rel : 0;
#pragma unroll
        for (int k = 0; k < kExactSums; ++k) {
          const float v = bperm(src, M[k]);
          tot[k] += mine ? v : 0.f;
        }
      }
      base += P;
    }
    if (uint32_t(lane) < m) {
      float4 *o = partials + 4 * uint64_t(slot);
      o[0] = make_float4(tot[0], tot[1], tot[2], tot[3]);
      o[1] = make_float4(tot[4], tot[5], tot[6], tot[7]);
      o[2] = make_float4(tot[8], tot[9], tot[10], tot[11]);
      o[3] = make_float4(tot[12], 0.f, 0.f, 0.f);
    }
    wave_lds_sync();
  }
}

// Ray-exact counterpart of record_grad_kernel: each record's 64-byte slots
// are reduced in order (groups of kGradLanes lanes, fixed butterfly), then
// exact_backward applies the chain rule.
__global__ __launch_bounds__(256) void record_grad_exact_kernel(fgs_gaussians g, GeomDev G,
                                                                const uint32_t *__restrict__ offset,
                                                                const float4 *__restrict__ partials, uint64_t R,
                                                                const uint32_t *__restrict__ kdev,
                                                                float *__restrict__ grad_rec) {
  __shared__ float s_sum[256][kExactSums + 1];
  const bool none = kdev[1] != 0u;
  const int t = threadIdx.x;
  const int64_t i0 = int64_t(blockIdx.x) * 256;
  const int v_local = blockIdx.y;
  const uint64_t rbase = uint64_t(v_local) * uint64_t(g.n);
  const int li = t % kGradLanes;
  for (int idx = t / kGradLanes; idx < 256; idx += 256 / kGradLanes) {
    float acc[kExactSums];
#pragma unroll
    for (int c = 0; c < kExactSums; ++c) acc[c] = 0.f;
    if (i0 + idx < g.n && !none) {
      const uint64_t r = rbase + uint64_t(i0 + idx);
      const uint32_t o = offset[r], end = offset[r + 1];
      for (uint32_t p = o + li; p < end; p += kGradLanes) {
        const float4 *q = partials + 4 * uint64_t(p);
        const float4 x0 = q[0], x1 = q[1], x2 = q[2];
        const float x3 = q[3].x;
        acc[0] += x0.x; acc[1] += x0.y; acc[2] += x0.z; acc[3] += x0.w;
        acc[4] += x1.x; acc[5] += x1.y; acc[6] += x1.z; acc[7] += x1.w;
        acc[8] += x2.x; acc[9] += x2.y; acc[10] += x2.z; acc[11] += x2.w;
        acc[12] += x3;
      }
    }
#pragma unroll
    for (int d = 1; d < kGradLanes; d <<= 1)
#pragma unroll
      for (int c = 0; c < kExactSums; ++c) acc[c] += __shfl_xor(acc[c], d, kGradLanes);
    if (li == 0)
#pragma unroll
      for (int c = 0; c < kExactSums; ++c) s_sum[idx][c] = acc[c];
  }
  __syncthreads();
  const int64_t i = i0 + t;
  if (i >= g.n) return;
  const uint64_t r = rbase + uint64_t(i);
  float out[11];
  bool zero = none || offset[r] == offset[r + 1];
  ExactSplat X;
  GaussParams P;
  ViewFrame F;
  if (!zero) {
    load_gauss(g, i, P);
    make_frame(G, G.view_begin + v_local, F);
    exact_forward(P, F, G, X);
    zero = !X.ok;
  }
  if (zero) {
#pragma unroll
    for (int c = 0; c < 11; ++c) grad_rec[uint64_t(c) * R + r] = 0.f;
    return;
  }
  float sums[kExactSums];
#pragma unroll
  for (int c = 0; c < kExactSums; ++c) sums[c] = s_sum[t][c];
  exact_backward(P, F, G, X, sums, out);
#pragma unroll
  for (int c = 0; c < 11; ++c) grad_rec[uint64_t(c) * R + r] = out[c];
}

// ------------------------------------------------------------------ host

struct RastLayout {
  uint64_t R, T, K;
  // byte offsets
  uint64_t total64, kdev, xy, radii, rect, offset, rec, scan_scratch, rng, grad_rec;
  uint64_t fixed_end;
  uint64_t keys, vals, keys_alt, vals_alt, sort_scratch, partials, ufirst, utile, uslots;
  uint64_t total, n_units;
  bool sorted_in_alt;
  int record_bits;  // > 0: one-word lists (tile << record_bits | record), no values arrays
};

// exact: the ray-exact model's 64-byte records and pair slots (else 32).
RastLayout rast_layout(uint64_t R, uint64_t T, uint64_t K, bool exact, int tile_bits) {
  RastLayout L{};
  L.R = R;
  L.T = T;
  L.K = K;
  Carver c(nullptr);
  c.take<unsigned long long>(1, &L.total64);
  c.take<uint32_t>(4, &L.kdev);
  c.take<float2>(R, &L.xy);
  c.take<float2>(R, &L.radii);
  c.take<ushort4>(R, &L.rect);
  c.take<uint32_t>(R + 1, &L.offset);
  if (exact)
    c.take<ExactRec>(R, &L.rec);
  else
    c.take<SplatRec>(R, &L.rec);
  c.take<uint32_t>(scan_scratch_words(R), &L.scan_scratch);
  c.take<uint2>(T, &L.rng);
  c.take<float>(11 * R, &L.grad_rec);
  L.fixed_end = c.used;
  // one-word lists when the tile field and the record index fit 32 bits
  // together (512^2 views: 10 + 22 bits, up to 4 M records per call): the
  // sort then moves 4 bytes per key and pass instead of 8
  const int rb = bits_for(R) > 0 ? bits_for(R) : 1;
  L.record_bits = tile_bits + rb <= 32 ? rb : 0;
  c.take<uint32_t>(K, &L.keys);
  c.take<uint32_t>(L.record_bits ? 0 : K, &L.vals);
  c.take<uint32_t>(K, &L.keys_alt);
  c.take<uint32_t>(L.record_bits ? 0 : K, &L.vals_alt);
  c.take<uint32_t>(sort_scratch_words(K), &L.sort_scratch);
  // per pair: the splat backward's six sums in a 32-byte slot (two aligned
  // 16-byte stores; 24-byte slots straddle lines and measured 1.5x the
  // backward's HBM writes, and a slower record gradient), the ray-exact
  // one's 13 in a 64-byte slot
  c.take<float>((exact ? 16 : 8) * K, &L.partials);
  L.n_units = units_bound(T, K);
  c.take<uint32_t>(T + 1, &L.ufirst);
  c.take<uint32_t>(L.n_units, &L.utile);
  // the forward's 16 x 16 partial sums per work unit (calls with few tiles)
  c.take<float>(!exact && chunks_per_tile(T) > 1 ? L.n_units * uint64_t(kTS * kTS) : 0, &L.uslots);
  L.total = c.used;
  const int bits = tile_bits;
  const int passes = sort_passes(K, bits, rast_sort_bits(K, bits));
  L.sorted_in_alt = (passes & 1) != 0;
  return L;
}

struct TileGrid {
  int tiles_x, tiles_y, tpv;
};

// Calls with few tiles split each list into work units (splat model) or a
// fixed number of strided chunks (ray-exact model); the forward keeps one
// partial image per piece index or chunk. Large calls take one wave per tile.
inline bool use_units(uint64_t T, bool exact) { return !exact && chunks_per_tile(T) > 1; }

// Bytes of the forward's partial images after the lists: one per chunk for
// the ray-exact model with few tiles (the splat model's units have slots in
// the lists' layout), none otherwise.
inline uint64_t forward_partial_bytes(uint64_t T, bool exact, uint64_t n_img) {
  const int c = chunks_per_tile(T);
  return (exact && c > 1) ? uint64_t(c) * n_img * sizeof(float) + 256 : 0;
}

template <typename T>
T *at(void *base, uint64_t off);

// The sorted lists' record indices in a workspace laid out by L.
ListRecs list_recs(const RastLayout &L, void *b) {
  if (L.record_bits)
    return ListRecs{at<uint32_t>(b, L.sorted_in_alt ? L.keys_alt : L.keys), (1u << L.record_bits) - 1u};
  return ListRecs{at<uint32_t>(b, L.sorted_in_alt ? L.vals_alt : L.vals), 0xffffffffu};
}

Units make_units(const RastLayout &L, void *b, bool on) {
  if (!on) return Units{nullptr, nullptr, 0u};
  return Units{at<uint32_t>(b, L.ufirst), at<uint32_t>(b, L.utile), uint32_t(L.n_units)};
}

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
  if (o->ablate & ~(FGS_ABLATE_SQUARE_BOX | FGS_ABLATE_QUADRANT_CULL | FGS_ABLATE_PER_PIXEL_BWD))
    return fail(FGS_E_INVALID, "unknown ablate bits");
  if (o->model != FGS_MODEL_SPLAT && o->model != FGS_MODEL_RAY_EXACT) return fail(FGS_E_INVALID, "opts.model");
  if (o->model == FGS_MODEL_RAY_EXACT && o->ablate)
    return fail(FGS_E_UNSUPPORTED, "the ablation switches apply to the splat model only");
  if (!(o->density_aabb_tau >= 0.f) || !std::isfinite(o->density_aabb_tau))
    return fail(FGS_E_INVALID, "density_aabb_tau must be finite and >= 0");
  if (o->density_aabb_tau > 0.f && (o->model == FGS_MODEL_RAY_EXACT || o->ablate))
    return fail(FGS_E_UNSUPPORTED, "the density-aware support applies to the splat model without ablation switches");
  return FGS_OK;
}

// The ray-exact kernels run for the ray-exact model in cone beam; in
// parallel beam the two models are the same function and the splat kernels run.
bool use_exact(const fgs_geom *geom, const fgs_opts *o) {
  return o->model == FGS_MODEL_RAY_EXACT && geom->mode == FGS_CONE;
}

ExactCam exact_cam(const GeomDev &G) {
  return ExactCam{G.fu, G.fv, G.cu, G.cv, G.kappa * G.kappa};
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
  G.tau = o->density_aabb_tau;
  G.ablate = o->ablate;
  G.angles = geom->angles;
  return G;
}

// Steps 1-5. On success the workspace holds records, sorted lists and tile
// starts; *Lout describes them.
// extra_bytes: room the caller needs after the lists (partial images).
int build_lists(const fgs_gaussians *g, const fgs_geom *geom, int32_t view_begin, int32_t view_count,
                const fgs_opts *o, fgs_workspace *ws, hipStream_t s, RastLayout *Lout,
                uint64_t extra_bytes = 0) {
  const uint64_t R = uint64_t(view_count) * uint64_t(g->n);
  const TileGrid tg = tile_grid(geom->det_w, geom->det_h);
  const uint64_t T = uint64_t(view_count) * uint64_t(tg.tpv);
  if (T >= 0xffffffffull || R >= 0xffffffffull) return fail(FGS_E_UNSUPPORTED, "too many tiles or records in one call");
  const bool exact = use_exact(geom, o);
  const int tile_bits = bits_for(uint64_t(tg.tpv));
  // key_capacity > 0: the lists are laid out for that many pairs and the
  // pair count stays on the device (no wait); else it is read back first
  const uint64_t cap = ws->key_capacity;
  if (cap >= 0xffffffffull) return fail(FGS_E_UNSUPPORTED, "key_capacity must be below 2^32");
  RastLayout L = rast_layout(R, T, cap, exact, tile_bits);
  ws->kind = 0;
  if (cap > 0) {
    ws->needed = L.total + extra_bytes;
    ws->n_pairs = cap;
    ws->n_records = R;
    ws->n_tiles = T;
    ws->tile_bits = tile_bits;
    ws->record_bits = L.record_bits;
    ws->n_gauss = uint64_t(g->n);
    if (!ws->ptr || ws->bytes < ws->needed) return fail(FGS_E_CAPACITY, "workspace too small for key_capacity pairs");
  } else if (!ws->ptr || ws->bytes < L.fixed_end + (uint64_t(1) << 20)) {
    ws->needed = L.fixed_end + (uint64_t(64) << 20);
    return fail(FGS_E_CAPACITY, "workspace too small for the per-record arrays");
  }
  GeomDev G = make_geom_dev(geom, o, view_begin, tg);
  void *b = ws->ptr;
  unsigned long long *total64 = at<unsigned long long>(b, L.total64);
  dim3 rgrid(grid_for(uint64_t(g->n), 256), unsigned(view_count));
  if (exact)
    record_kernel<true><<<rgrid, 256, 0, s>>>(*g, G, at<float2>(b, L.xy), at<void>(b, L.rec),
                                              at<float2>(b, L.radii), at<ushort4>(b, L.rect),
                                              at<uint32_t>(b, L.offset));
  else
    record_kernel<false><<<rgrid, 256, 0, s>>>(*g, G, at<float2>(b, L.xy), at<void>(b, L.rec),
                                               at<float2>(b, L.radii), at<ushort4>(b, L.rect),
                                               at<uint32_t>(b, L.offset));
  FGS_LAUNCH_CHECK("record_kernel");
  // offsets, the 64-bit pair total and the device pair count (0 past the
  // capacity) in one scan
  uint32_t *kdev = at<uint32_t>(b, L.kdev);
  int st = scan_counts(at<uint32_t>(b, L.offset), R, at<uint32_t>(b, L.scan_scratch),
                       cap > 0 ? cap : uint64_t(0xfffffffeull), total64, kdev, cap > 0 ? ws->overflow : nullptr, s);
  if (st != FGS_OK) return st;
  if (cap == 0) {
    unsigned long long K64 = 0;
    FGS_HIP(hipMemcpyAsync(&K64, total64, sizeof(K64), hipMemcpyDeviceToHost, s));
    FGS_HIP(hipStreamSynchronize(s));
    if (K64 >= 0xffffffffull)
      return fail(FGS_E_UNSUPPORTED, "more than 2^32 (tile, Gaussian) pairs in one call; split the views");
    const uint64_t K = K64;
    L = rast_layout(R, T, K, exact, tile_bits);
    ws->needed = L.total + extra_bytes;
    ws->n_pairs = K;
    ws->n_records = R;
    ws->n_tiles = T;
    ws->tile_bits = tile_bits;
    ws->record_bits = L.record_bits;
    ws->n_gauss = uint64_t(g->n);
    if (ws->bytes < L.total + extra_bytes) return fail(FGS_E_CAPACITY, "workspace too small for the tile lists");
  }
  if (L.K > 0) {
    auto emit = [&](auto rpb) {
      constexpr int RPB = decltype(rpb)::value;
      emit_kernel<RPB><<<grid_for(R, RPB), kEmitBlock, 0, s>>>(R, g->n, tg.tiles_x, tile_bits, L.record_bits,
          at<ushort4>(b, L.rect),
          at<uint32_t>(b, L.offset), at<uint32_t>(b, L.keys),
          L.record_bits ? nullptr : at<uint32_t>(b, L.vals),
          exact ? &at<ExactRec>(b, L.rec)->d.y : &at<SplatRec>(b, L.rec)->b.z,
          exact ? 16u : 8u, kdev);
    };
    // a call of fewer than 256 K records: 64 records per block
    if (R < (uint64_t(1) << 18))
      emit(std::integral_constant<int, 64>());
    else
      emit(std::integral_constant<int, kEmitBlock>());
    FGS_LAUNCH_CHECK("emit_kernel");
  }
  uint32_t *sk, *sv;
  st = radix_sort_pairs(at<uint32_t>(b, L.keys), L.record_bits ? nullptr : at<uint32_t>(b, L.vals),
                        at<uint32_t>(b, L.keys_alt), L.record_bits ? nullptr : at<uint32_t>(b, L.vals_alt), L.K,
                        tile_bits, at<uint32_t>(b, L.sort_scratch), &sk, &sv, s, rast_sort_bits(L.K, tile_bits),
                        cap > 0 ? kdev : nullptr, L.record_bits);
  if (st != FGS_OK) return st;
  if (L.K > 0) {
    const uint64_t waves = (L.K + uint64_t(kWave * kRangeItems) - 1) / uint64_t(kWave * kRangeItems);
    ranges_kernel<<<grid_for(waves * kWave, 256), 256, 0, s>>>(sk, L.K, kdev, tile_bits, uint32_t(tg.tpv),
                                                               L.record_bits, uint32_t(g->n), T, at<uint2>(b, L.rng));
    FGS_LAUNCH_CHECK("ranges_kernel");
  } else {
    zero_ranges_kernel<<<grid_for(T, 256), 256, 0, s>>>(at<uint2>(b, L.rng), T);
    FGS_LAUNCH_CHECK("zero_ranges_kernel");
  }
  if (use_units(T, exact)) {
    unit_offsets_kernel<<<1, 1024, 0, s>>>(at<uint2>(b, L.rng), uint32_t(T), uint32_t(L.n_units),
                                           at<uint32_t>(b, L.ufirst), at<uint32_t>(b, L.utile));
    FGS_LAUNCH_CHECK("unit_offsets_kernel");
  }
  ws->kind = exact ? 3 : 1;
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
  const TileGrid tg = tile_grid(geom->det_w, geom->det_h);
  const uint64_t T = uint64_t(view_count) * uint64_t(tg.tpv);
  const bool exact = use_exact(geom, opts);
  const int chunks = chunks_per_tile(T);
  const uint64_t n_img = uint64_t(view_count) * uint64_t(geom->det_w) * uint64_t(geom->det_h);
  // the ray-exact model's partial images of the chunks, after the lists
  const uint64_t part_bytes = forward_partial_bytes(T, exact, n_img);
  RastLayout L;
  st = build_lists(g, geom, view_begin, view_count, opts, ws, s, &L, part_bytes);
  if (st != FGS_OK) return st;
  void *b = ws->ptr;
  float *part = part_bytes ? at<float>(b, (L.total + 255) / 256 * 256)
                           : (use_units(T, exact) ? at<float>(b, L.uslots) : img);
  const ListRecs sv = list_recs(L, b);
  const float thr = -0.5f * kLog2e * opts->kappa * opts->kappa;
  const float log2_tau = opts->density_aabb_tau > 0.f ? log2f(opts->density_aabb_tau) : -INFINITY;
  hipEvent_t *ev = static_cast<hipEvent_t *>(opts->events);
  if (ev) FGS_HIP(hipEventRecord(ev[0], s));
  if (exact) {
    const uint64_t units = L.T * uint64_t(chunks);
    const ExactCam cam = exact_cam(make_geom_dev(geom, opts, view_begin, tg));
    with_tiles_per_block(units, [&](auto tpb) {
      constexpr int TPB = decltype(tpb)::value;
      splat_fwd_exact_kernel<false, TPB><<<grid_for(units, TPB), kWave * TPB, 0, s>>>(
          at<uint2>(b, L.rng), sv, at<ExactRec>(b, L.rec), tg.tiles_x, tg.tpv, geom->det_w, geom->det_h,
          uint32_t(L.T), chunks, thr, thr * kCullSlack, cam, part, nullptr);
    });
    FGS_LAUNCH_CHECK("splat_fwd_exact_kernel");
    if (part_bytes) {
      st = sum_chunks(part, chunks, n_img, img, s);
      if (st != FGS_OK) return st;
    }
  } else {
    const Units U = make_units(L, b, use_units(T, false));
    const uint64_t units = U.first ? L.n_units : L.T;
    const int no_cull = (opts->ablate & FGS_ABLATE_QUADRANT_CULL) ? 1 : 0;
    const bool interior = L.K >= kInteriorKeysPerRecord * L.R;
    const bool tau = opts->density_aabb_tau > 0.f;
    with_tiles_per_block(units, [&](auto tpb) {
      constexpr int TPB = decltype(tpb)::value;
      if (tau)
        splat_fwd_kernel<false, false, TPB, true><<<grid_for(units, TPB), kWave * TPB, 0, s>>>(
            at<uint2>(b, L.rng), sv, at<SplatRec>(b, L.rec), tg.tiles_x, tg.tpv, geom->det_w, geom->det_h,
            uint32_t(L.T), 1, U, thr, log2_tau, no_cull, part, nullptr);
      else if (interior)
        splat_fwd_kernel<false, true, TPB, false><<<grid_for(units, TPB), kWave * TPB, 0, s>>>(
            at<uint2>(b, L.rng), sv, at<SplatRec>(b, L.rec), tg.tiles_x, tg.tpv, geom->det_w, geom->det_h,
            uint32_t(L.T), 1, U, thr, log2_tau, no_cull, part, nullptr);
      else
        splat_fwd_kernel<false, false, TPB, false><<<grid_for(units, TPB), kWave * TPB, 0, s>>>(
            at<uint2>(b, L.rng), sv, at<SplatRec>(b, L.rec), tg.tiles_x, tg.tpv, geom->det_w, geom->det_h,
            uint32_t(L.T), 1, U, thr, log2_tau, no_cull, part, nullptr);
    }, L.K >= kSmallBlockKeysPerTile * L.T);
    FGS_LAUNCH_CHECK("splat_fwd_kernel");
    if (U.first) {
      sum_units_kernel<<<grid_for(n_img, 256), 256, 0, s>>>(part, U.first, tg.tiles_x, tg.tpv, geom->det_w,
                                                             geom->det_h, n_img, img);
      FGS_LAUNCH_CHECK("sum_units_kernel");
    }
  }
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
  zero_u64_kernel<<<1, 1, 0, s>>>(cnt, 1);
  FGS_LAUNCH_CHECK("zero_u64_kernel");
  const ListRecs sv = list_recs(L, b);
  const float thr = -0.5f * kLog2e * opts->kappa * opts->kappa;
  const float log2_tau = opts->density_aabb_tau > 0.f ? log2f(opts->density_aabb_tau) : -INFINITY;
  const TileGrid tg = tile_grid(geom->det_w, geom->det_h);
  const int chunks = chunks_per_tile(L.T);
  const uint64_t units = L.T * uint64_t(chunks);
  if (use_exact(geom, opts)) {
    const ExactCam cam = exact_cam(make_geom_dev(geom, opts, view_begin, tg));
    with_tiles_per_block(units, [&](auto tpb) {
      constexpr int TPB = decltype(tpb)::value;
      splat_fwd_exact_kernel<true, TPB><<<grid_for(units, TPB), kWave * TPB, 0, s>>>(
          at<uint2>(b, L.rng), sv, at<ExactRec>(b, L.rec), tg.tiles_x, tg.tpv, geom->det_w, geom->det_h,
          uint32_t(L.T), chunks, thr, thr * kCullSlack, cam, nullptr, cnt);
    });
    FGS_LAUNCH_CHECK("splat_fwd_exact_kernel<count>");
    return FGS_OK;
  }
  const Units U = make_units(L, b, use_units(L.T, false));
  const uint64_t sunits = U.first ? L.n_units : L.T;
  with_tiles_per_block(sunits, [&](auto tpb) {
    constexpr int TPB = decltype(tpb)::value;
    if (opts->density_aabb_tau > 0.f)
      splat_fwd_kernel<true, false, TPB, true><<<grid_for(sunits, TPB), kWave * TPB, 0, s>>>(
          at<uint2>(b, L.rng), sv, at<SplatRec>(b, L.rec), tg.tiles_x, tg.tpv, geom->det_w, geom->det_h,
          uint32_t(L.T), 1, U, thr, log2_tau, 0, nullptr, cnt);
    else
      splat_fwd_kernel<true, false, TPB, false><<<grid_for(sunits, TPB), kWave * TPB, 0, s>>>(
          at<uint2>(b, L.rng), sv, at<SplatRec>(b, L.rec), tg.tiles_x, tg.tpv, geom->det_w, geom->det_h,
          uint32_t(L.T), 1, U, thr, log2_tau, 0, nullptr, cnt);
  }, L.K >= kSmallBlockKeysPerTile * L.T);
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
    if (ws->kind != (use_exact(geom, opts) ? 3 : 1) || ws->n_records != R || !ws->ptr)
      return fail(FGS_E_INVALID, "workspace does not hold this call's rasterizer lists");
    const uint64_t T = uint64_t(view_count) * uint64_t(tile_grid(geom->det_w, geom->det_h).tpv);
    L = rast_layout(R, T, ws->n_pairs, use_exact(geom, opts), ws->tile_bits);
    if (T != ws->n_tiles || ws->bytes < L.total)
      return fail(FGS_E_INVALID, "workspace lists do not match this call");
  }
  void *b = ws->ptr;
  const TileGrid tg = tile_grid(geom->det_w, geom->det_h);
  GeomDev G = make_geom_dev(geom, opts, view_begin, tg);
  const ListRecs sv = list_recs(L, b);
  const float thr = -0.5f * kLog2e * opts->kappa * opts->kappa;
  const float log2_tau = opts->density_aabb_tau > 0.f ? log2f(opts->density_aabb_tau) : -INFINITY;
  hipEvent_t *ev = static_cast<hipEvent_t *>(opts->events);
  if (ev) FGS_HIP(hipEventRecord(ev[0], s));
  if (use_exact(geom, opts)) {
    if (L.K > 0) {
      const int chunks = chunks_per_tile(L.T);
      const uint64_t units = L.T * uint64_t(chunks);
      const ExactCam cam = exact_cam(G);
      with_tiles_per_block(units, [&](auto tpb) {
        constexpr int TPB = decltype(tpb)::value;
        splat_bwd_exact_kernel<TPB><<<grid_for(units, TPB), kWave * TPB, 0, s>>>(
            at<uint2>(b, L.rng), sv, at<ExactRec>(b, L.rec), tg.tiles_x, tg.tpv, geom->det_w, geom->det_h,
            uint32_t(L.T), chunks, thr, thr * kCullSlack, cam, grad_img, at<float4>(b, L.partials));
      }, true);
      FGS_LAUNCH_CHECK("splat_bwd_exact_kernel");
    }
    if (ev) FGS_HIP(hipEventRecord(ev[1], s));
    dim3 rgrid(grid_for(uint64_t(g->n), 256), unsigned(view_count));
    record_grad_exact_kernel<<<rgrid, 256, 0, s>>>(*g, G, at<uint32_t>(b, L.offset), at<float4>(b, L.partials), R,
                                                   at<uint32_t>(b, L.kdev), at<float>(b, L.grad_rec));
    FGS_LAUNCH_CHECK("record_grad_exact_kernel");
    view_sum_kernel<<<grid_for(uint64_t(g->n), 256), 256, 0, s>>>(g->n, view_count, at<float>(b, L.grad_rec),
                                                                  *out, opts->accumulate);
    FGS_LAUNCH_CHECK("view_sum_kernel");
    return FGS_OK;
  }
  float *acc6 = nullptr;
  if (opts->ablate & FGS_ABLATE_PER_PIXEL_BWD) {
    // the records' accumulators take the place of the pair slots
    if (L.K < R) return fail(FGS_E_UNSUPPORTED, "per-pixel backward ablation: too few pairs");
    acc6 = at<float>(b, L.partials);
    fill_zero_kernel<<<grid_for(6 * R, 256), 256, 0, s>>>(acc6, 6 * R);
    FGS_LAUNCH_CHECK("fill_zero_kernel");
    if (L.K > 0) {
      splat_bwd_pixel_kernel<<<unsigned(L.T), kWave, 0, s>>>(at<uint2>(b, L.rng), sv, at<SplatRec>(b, L.rec),
                                                             tg.tiles_x, tg.tpv, geom->det_w, geom->det_h,
                                                             uint32_t(L.T), thr, grad_img, acc6);
      FGS_LAUNCH_CHECK("splat_bwd_pixel_kernel");
    }
  } else if (L.K > 0) {
    const Units U = make_units(L, b, use_units(L.T, false));
    const int chunks = U.first ? 1 : chunks_per_tile(L.T);
    const uint64_t units = U.first ? L.n_units : L.T * uint64_t(chunks);
    with_tiles_per_block(units, [&](auto tpb) {
      constexpr int TPB = decltype(tpb)::value;
      if (opts->density_aabb_tau > 0.f)
        splat_bwd_kernel<TPB, true><<<grid_for(units, TPB), kWave * TPB, 0, s>>>(
            at<uint2>(b, L.rng), sv, at<SplatRec>(b, L.rec), tg.tiles_x, tg.tpv, geom->det_w, geom->det_h,
            uint32_t(L.T), chunks, U, thr, log2_tau, (opts->ablate & FGS_ABLATE_QUADRANT_CULL) ? 1 : 0,
            grad_img, at<float4>(b, L.partials));
      else
        splat_bwd_kernel<TPB, false><<<grid_for(units, TPB), kWave * TPB, 0, s>>>(
            at<uint2>(b, L.rng), sv, at<SplatRec>(b, L.rec), tg.tiles_x, tg.tpv, geom->det_w, geom->det_h,
            uint32_t(L.T), chunks, U, thr, log2_tau, (opts->ablate & FGS_ABLATE_QUADRANT_CULL) ? 1 : 0,
            grad_img, at<float4>(b, L.partials));
    }, true);
    FGS_LAUNCH_CHECK("splat_bwd_kernel");
  }
  if (ev) FGS_HIP(hipEventRecord(ev[1], s));
  // few records (one view): 64 records per block, so that the blocks cover
  // the chip; the sums are the same either way
  // one view: the records' gradients go straight to the output (the sum
  // over one view is the identity), without view_sum_kernel
  const GradSink sink{at<float>(b, L.grad_rec), R, *out, opts->accumulate};
  const bool direct = view_count == 1;
  auto launch = [&](auto rpb, auto dir) {
    constexpr int RPB = decltype(rpb)::value;
    dim3 rgrid(grid_for(uint64_t(g->n), RPB), unsigned(view_count));
    record_grad_kernel<RPB, decltype(dir)::value><<<rgrid, 256, 0, s>>>(
        *g, G, at<uint32_t>(b, L.offset), at<float4>(b, L.partials), acc6, R, at<uint32_t>(b, L.kdev), sink);
  };
  using I64 = std::integral_constant<int, 64>;
  using I256 = std::integral_constant<int, 256>;
  if (uint64_t(grid_for(uint64_t(g->n), 256)) * uint64_t(view_count) < 2048) {
    if (direct) launch(I64(), std::true_type()); else launch(I64(), std::false_type());
  } else {
    if (direct) launch(I256(), std::true_type()); else launch(I256(), std::false_type());
  }
  FGS_LAUNCH_CHECK("record_grad_kernel");
  if (view_count > 1) {
    view_sum_kernel<<<grid_for(uint64_t(g->n), 256), 256, 0, s>>>(g->n, view_count, at<float>(b, L.grad_rec),
                                                                  *out, opts->accumulate);
    FGS_LAUNCH_CHECK("view_sum_kernel");
  }
  return FGS_OK;
}

namespace fgs {
// Workspace of a rasterizer call over R records and T tiles: bytes that do
// not depend on the number of (tile, Gaussian) pairs K, and an upper bound
// on the bytes per pair (fixed + K * per_key covers every K). The forward of
// a call with few tiles also keeps one partial image per chunk.
int rast_workspace_bytes(const fgs_gaussians *g, const fgs_geom *geom, int32_t view_count, const fgs_opts *o,
                         bool forward, uint64_t *fixed_bytes, uint64_t *bytes_per_key) {
  if (!g || !geom || !o || g->n <= 0 || view_count <= 0 || view_count > geom->n_views || geom->det_w <= 0 ||
      geom->det_h <= 0)
    return fail(FGS_E_INVALID, "workspace query: null argument, no Gaussians, detector size or view count");
  if (o->model != FGS_MODEL_SPLAT && o->model != FGS_MODEL_RAY_EXACT) return fail(FGS_E_INVALID, "opts.model");
  const TileGrid tg = tile_grid(geom->det_w, geom->det_h);
  const uint64_t R = uint64_t(view_count) * uint64_t(g->n);
  const uint64_t T = uint64_t(view_count) * uint64_t(tg.tpv);
  const bool exact = use_exact(geom, o);
  const int bits = bits_for(uint64_t(tg.tpv));
  const uint64_t k_ref = uint64_t(1) << 24;
  const uint64_t base = rast_layout(R, T, 0, exact, bits).total;
  const uint64_t big = rast_layout(R, T, k_ref, exact, bits).total;
  const uint64_t n_img = uint64_t(view_count) * uint64_t(geom->det_w) * uint64_t(geom->det_h);
  const uint64_t part = forward ? forward_partial_bytes(T, exact, n_img) : 0;
  // every array the pair count sizes is padded to 256 bytes: 8 arrays at most
  // (a call first asks for the per-record arrays plus 1 MiB before it knows K)
  *fixed_bytes = base + part + 8 * kAlign + (uint64_t(1) << 20);
  *bytes_per_key = (big - base + k_ref - 1) / k_ref;
  return FGS_OK;
}

int rast_binning_layout(const fgs_workspace *ws, uint64_t off[9], uint64_t counts[3]) {
  RastLayout L = rast_layout(ws->n_records, ws->n_tiles, ws->n_pairs, ws->kind == 3, ws->tile_bits);
  off[0] = L.xy;
  off[1] = L.radii;
  off[2] = L.rect;
  off[3] = L.offset;
  // one-word lists (ws->record_bits > 0) have no values arrays: the value
  // offsets repeat the key offsets (the words hold both)
  off[4] = L.sorted_in_alt ? L.keys : L.keys_alt;
  off[5] = L.record_bits ? off[4] : (L.sorted_in_alt ? L.vals : L.vals_alt);
  off[6] = L.sorted_in_alt ? L.keys_alt : L.keys;
  off[7] = L.record_bits ? off[6] : (L.sorted_in_alt ? L.vals_alt : L.vals);
  off[8] = L.rng;
  counts[0] = L.R;
  counts[1] = L.K;
  counts[2] = L.T;
  return FGS_OK;
}
}  // namespace fgs
