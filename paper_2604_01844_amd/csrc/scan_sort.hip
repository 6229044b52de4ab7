// Device-wide exclusive scan and stable LSD radix sort of uint32 (key, value)
// pairs, written for 64-wide wavefronts.
//
// The rasterizer and voxelizer bin Gaussians into tiles without any depth
// ordering (the X-ray sum is order-free, Sec. 3.5): the sort key is only the
// (view, tile) index. Keys are emitted in record order, so a stable sort
// leaves each tile's list in ascending Gaussian index, which fixes the
// summation order and makes every result bit-reproducible.
//
// Scan: reduce-then-scan over tiles of 4096 values (256 threads x 16).
// Sort: per pass of up to 9 key bits, (1) a per-tile digit histogram in LDS,
// (2) an exclusive scan of the digit-major histogram table, (3) a scatter in
// which every wave ranks its keys with ballot-based digit matching (64-bit
// lane masks), so the local order of equal digits is the input order.
#include "fgs_internal.h"

namespace fgs {
namespace {

constexpr int kThreads = 256;
constexpr int kItems = 16;
constexpr int kTile = kThreads * kItems;  // 4096
constexpr int kWaves = kThreads / 64;
constexpr int kMaxBins = 1 << kSortMaxBits;
// Scans of at most this many tiles of kTile values let each block sum the
// tile totals before it instead of scanning them in a launch of their own.
constexpr uint64_t kSelfPrefixTiles = 4096;

// Exclusive scan of one value per thread across the 256-thread block.
template <typename T>
__device__ __forceinline__ T block_exclusive_scan(T v, T *wsum, T &total) {
  const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
  T x = v;
#pragma unroll
  for (int d = 1; d < 64; d <<= 1) {
    T y = __shfl_up(x, d, 64);
    if (lane >= d) x += y;
  }
  if (lane == 63) wsum[wid] = x;
  __syncthreads();
  T base = 0, tot = 0;
#pragma unroll
  for (int w = 0; w < kWaves; ++w) {
    T s = wsum[w];
    base += (w < wid) ? s : T(0);
    tot += s;
  }
  total = tot;
  __syncthreads();
  return base + x - v;
}

template <typename T>
__global__ __launch_bounds__(kThreads) void scan_reduce_kernel(const T *__restrict__ data, uint64_t n,
                                                               T *__restrict__ partial) {
  __shared__ T wsum[kWaves];
  const uint64_t base = uint64_t(blockIdx.x) * kTile;
  T s = 0;
#pragma unroll
  for (int j = 0; j < kItems; ++j) {
    uint64_t idx = base + uint64_t(j) * kThreads + threadIdx.x;
    s += (idx < n) ? data[idx] : T(0);
  }
  T total;
  block_exclusive_scan(s, wsum, total);
  if (threadIdx.x == 0) partial[blockIdx.x] = total;
}

// The pair count of a binning, taken from the scan of its per-record key
// counts (count == null: none). total: the 64-bit sum of the counts;
// count[0] = that sum if it is at most cap, else 0 (nothing is binned);
// count[1] = 1 if it exceeds cap, else 0; with a non-null overflow (device
// uint32[2]) an excess also sets overflow[0] = 1 and raises overflow[1] to
// the sum (clamped to 2^32 - 1).
struct CountOut {
  uint64_t cap;
  unsigned long long *total;
  uint32_t *count;
  uint32_t *overflow;
};

__device__ __forceinline__ void write_count(const CountOut &co, unsigned long long v) {
  const bool over = v > co.cap;
  co.total[0] = v;
  co.count[0] = over ? 0u : uint32_t(v);
  co.count[1] = over ? 1u : 0u;
  if (over && co.overflow) {
    co.overflow[0] = 1u;
    atomicMax(co.overflow + 1, uint32_t(v < 0xffffffffull ? v : 0xffffffffull));
  }
}

// Scans one tile in LDS; adds the tile's offset. partial (may be null for a
// single tile): with self_prefix, the tiles' sums, of which each block adds
// up those before it (one launch fewer; used for few tiles); else the
// already scanned tile offsets. The last tile writes the grand total to
// data[n] and, with co.count, the 64-bit total and the pair count: it adds
// up every tile's sum in 64 bits (a scanned offset table gives them as
// differences of neighbours, exact while one tile's sum fits 32 bits), so
// a 32-bit wrap of the offsets is detected.
template <typename T>
__global__ __launch_bounds__(kThreads) void scan_apply_kernel(T *__restrict__ data, uint64_t n,
                                                              const T *__restrict__ partial,
                                                              uint32_t n_tiles, int self_prefix, CountOut co) {
  __shared__ T tile[kTile + kTile / 32];
  __shared__ T wsum[kWaves];
  __shared__ T s_pre;
  __shared__ unsigned long long s_before64;
  const uint64_t base = uint64_t(blockIdx.x) * kTile;
  if (partial && self_prefix) {
    T acc = 0;
    for (uint32_t k = threadIdx.x; k < blockIdx.x; k += kThreads) acc += partial[k];
    T tot;
    block_exclusive_scan(acc, wsum, tot);
    if (threadIdx.x == 0) s_pre = tot;
    __syncthreads();
  }
  const bool count_here = co.count && blockIdx.x == n_tiles - 1;
  if (count_here) {
    // 64-bit sum of the tiles before this one
    __shared__ unsigned long long w64[kWaves];
    unsigned long long a64 = 0;
    if (partial)
      for (uint32_t k = threadIdx.x; k < blockIdx.x; k += kThreads)
        a64 += self_prefix ? (unsigned long long)partial[k] : (unsigned long long)T(partial[k + 1] - partial[k]);
    unsigned long long tot64;
    block_exclusive_scan(a64, w64, tot64);
    if (threadIdx.x == 0) s_before64 = tot64;
    __syncthreads();
  }
  // padded index: one spare word every 32 to spread the strided reads over banks
  auto pad = [](int i) { return i + (i >> 5); };
#pragma unroll
  for (int j = 0; j < kItems; ++j) {
    int li = j * kThreads + threadIdx.x;
    uint64_t idx = base + li;
    tile[pad(li)] = (idx < n) ? data[idx] : T(0);
  }
  __syncthreads();
  T v[kItems];
  T s = 0;
#pragma unroll
  for (int j = 0; j < kItems; ++j) {
    v[j] = tile[pad(threadIdx.x * kItems + j)];
    s += v[j];
  }
  T total;
  T run = block_exclusive_scan(s, wsum, total);
  const T off = partial ? (self_prefix ? s_pre : partial[blockIdx.x]) : T(0);
#pragma unroll
  for (int j = 0; j < kItems; ++j) {
    tile[pad(threadIdx.x * kItems + j)] = run + off;
    run += v[j];
  }
  __syncthreads();
#pragma unroll
  for (int j = 0; j < kItems; ++j) {
    int li = j * kThreads + threadIdx.x;
    uint64_t idx = base + li;
    if (idx < n) data[idx] = tile[pad(li)];
  }
  if (blockIdx.x == n_tiles - 1 && threadIdx.x == 0) {
    data[n] = off + total;
    if (count_here) write_count(co, s_before64 + (unsigned long long)total);
  }
}

// ------------------------------------------------------------- radix sort

// NB: the widest digit the kernel is built for (its LDS tables hold 2^NB
// bins); each pass runs the smallest build (6, 9 or 10 bits) that holds its
// digit, which needs the least LDS.
// n_dev (may be null): the number of pairs on the device, at most n; the
// grid is sized for n and tiles past the device count hold nothing.
__device__ __forceinline__ uint64_t pair_count(uint64_t n, const uint32_t *n_dev) {
  return n_dev ? min(n, uint64_t(*n_dev)) : n;
}

template <int NB>
__global__ __launch_bounds__(kThreads) void rs_hist_kernel(const uint32_t *__restrict__ keys,
                                                           uint64_t n_cap, const uint32_t *__restrict__ n_dev,
                                                           int shift, uint32_t mask,
                                                           uint32_t *__restrict__ hist,
                                                           uint32_t n_tiles) {
  constexpr int kBins = 1 << NB;
  __shared__ uint32_t h[kBins];
  const uint64_t n = pair_count(n_cap, n_dev);
  for (int i = threadIdx.x; i < kBins; i += kThreads) h[i] = 0;
  __syncthreads();
  const uint64_t base = uint64_t(blockIdx.x) * kTile;
  // all of the thread's loads first, so their latencies overlap
  uint32_t kk[kItems];
#pragma unroll
  for (int j = 0; j < kItems; ++j) {
    const uint64_t idx = base + uint64_t(j) * kThreads + threadIdx.x;
    kk[j] = idx < n ? keys[idx] : 0u;
  }
#pragma unroll
  for (int j = 0; j < kItems; ++j) {
    const uint64_t idx = base + uint64_t(j) * kThreads + threadIdx.x;
    if (idx < n) atomicAdd(&h[(kk[j] >> shift) & mask], 1u);
  }
  __syncthreads();
  for (uint32_t d = threadIdx.x; d <= mask; d += kThreads) hist[uint64_t(d) * n_tiles + blockIdx.x] = h[d];
}

// Stable scatter of one pass. Tile t covers input [t*4096, t*4096 + 4096);
// wave w of the tile owns the contiguous quarter [w*1024, w*1024 + 1024),
// processed 64 keys at a time, so (wave, round, lane) order is input order.
// Keys are first placed in LDS in the tile's digit-sorted order, then
// written out linearly: consecutive threads write consecutive positions of
// each digit's run, so the global writes are coalesced. kVals = false: keys
// only (the values arrays are not touched).
template <int NB, bool kVals>
__global__ __launch_bounds__(kThreads) void rs_scatter_kernel(
    const uint32_t *__restrict__ keys_in, const uint32_t *__restrict__ vals_in, uint64_t n_cap,
    const uint32_t *__restrict__ n_dev, int shift, int nbits, const uint32_t *__restrict__ hist_scanned,
    uint32_t n_tiles, uint32_t *__restrict__ keys_out, uint32_t *__restrict__ vals_out) {
  const uint64_t n = pair_count(n_cap, n_dev);
  // a tile past the device count (a grid sized for the capacity) moves nothing
  if (uint64_t(blockIdx.x) * kTile >= n) return;
  constexpr int kBins = 1 << NB;
  __shared__ uint32_t cnt[kWaves][kBins];
  __shared__ uint32_t s_local[kBins];     // tile-local start of each digit's run
  __shared__ uint32_t s_global[kBins];    // global start of each digit's run for this tile
  __shared__ uint32_t s_keys[kTile];
  __shared__ uint32_t s_vals[kVals ? kTile : 1];
  __shared__ uint32_t s_wsum[kWaves];
  const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
  const uint32_t mask = (1u << nbits) - 1u;
  for (int i = threadIdx.x; i < kWaves * kBins; i += kThreads) (&cnt[0][0])[i] = 0;
  __syncthreads();

  const uint64_t wbase = uint64_t(blockIdx.x) * kTile + uint64_t(wid) * (kItems * 64);
  const uint64_t lt_mask = (lane == 0) ? 0ull : (~0ull >> (64 - lane));
  uint32_t k[kItems], v[kItems], rank[kItems];
  // all of the wave's loads first, so their latencies overlap
#pragma unroll
  for (int j = 0; j < kItems; ++j) {
    const uint64_t idx = wbase + uint64_t(j) * 64 + lane;
    k[j] = idx < n ? keys_in[idx] : 0u;
    v[j] = (kVals && idx < n) ? vals_in[idx] : 0u;
  }
#pragma unroll
  for (int j = 0; j < kItems; ++j) {
    const uint64_t idx = wbase + uint64_t(j) * 64 + lane;
    const bool valid = idx < n;
    const uint32_t key = k[j];
    const uint32_t d = (key >> shift) & mask;
    uint64_t peers = __ballot(valid);
    for (int b = 0; b < nbits; ++b) {
      const bool bit = (d >> b) & 1u;
      const uint64_t m = __ballot(bit);
      peers &= bit ? m : ~m;
    }
    const uint32_t before = __popcll(peers & lt_mask);
    uint32_t c = 0;
    if (valid) c = cnt[wid][d];
    // the lowest lane of each digit group advances the wave's running count
    if (valid && before == 0) cnt[wid][d] = c + __popcll(peers);
    rank[j] = c + before;
  }
  __syncthreads();
  // per digit d: the tile's count, the waves' offsets inside the digit's run,
  // then an exclusive scan of the counts over digits (the tile-local starts)
  const int bins = int(mask) + 1;
  constexpr int kPer = (kBins + kThreads - 1) / kThreads;
  const int per_thread = (bins + kThreads - 1) / kThreads;  // <= kPer
  uint32_t tot[kPer] = {}, gstart[kPer] = {};
#pragma unroll
  for (int q = 0; q < kPer; ++q) {  // the table loads first, so they overlap
    const int d = threadIdx.x * per_thread + q;
    if (q < per_thread && d < bins) gstart[q] = hist_scanned[uint64_t(d) * n_tiles + blockIdx.x];
  }
#pragma unroll
  for (int q = 0; q < kPer; ++q) {
    const int d = threadIdx.x * per_thread + q;
    if (q < per_thread && d < bins) {
      uint32_t run = 0;
#pragma unroll
      for (int w = 0; w < kWaves; ++w) {
        const uint32_t c = cnt[w][d];
        cnt[w][d] = run;
        run += c;
      }
      tot[q] = run;
      s_global[d] = gstart[q];
    }
  }
  uint32_t mine = 0;
#pragma unroll
  for (int q = 0; q < kPer; ++q) mine += tot[q];
  uint32_t incl = mine;  // inclusive scan of `mine` over the block
  for (int o = 1; o < 64; o <<= 1) {
    const uint32_t y = __shfl_up(incl, o, 64);
    if (lane >= o) incl += y;
  }
  if (lane == 63) s_wsum[wid] = incl;
  __syncthreads();
  uint32_t excl = incl - mine;
  for (int w = 0; w < wid; ++w) excl += s_wsum[w];
  for (int q = 0; q < per_thread; ++q) {
    const int d = threadIdx.x * per_thread + q;
    if (d < bins) s_local[d] = excl;
    excl += tot[q];
  }
  __syncthreads();
#pragma unroll
  for (int j = 0; j < kItems; ++j) {
    const uint64_t idx = wbase + uint64_t(j) * 64 + lane;
    if (idx < n) {
      const uint32_t d = (k[j] >> shift) & mask;
      const uint32_t lp = s_local[d] + cnt[wid][d] + rank[j];
      s_keys[lp] = k[j];
      if (kVals) s_vals[lp] = v[j];
    }
  }
  __syncthreads();
  const uint64_t tbase = uint64_t(blockIdx.x) * kTile;
  const int nt = tbase < n ? int(min(uint64_t(kTile), n - tbase)) : 0;
  for (int i = threadIdx.x; i < nt; i += kThreads) {
    const uint32_t key = s_keys[i];
    const uint32_t d = (key >> shift) & mask;
    const uint32_t pos = s_global[d] + (uint32_t(i) - s_local[d]);
    keys_out[pos] = key;
    if (kVals) vals_out[pos] = s_vals[i];
  }
}

template <typename T>
__global__ void set_zero_kernel(T *p, CountOut co) {
  *p = T(0);
  if (co.count) write_count(co, 0ull);
}

}  // namespace

uint64_t scan_scratch_words(uint64_t n) {
  // in units of 64-bit words, enough for both element widths
  uint64_t words = 0;
  uint64_t m = n;
  while (m > uint64_t(kTile)) {
    uint64_t tiles = (m + kTile - 1) / kTile;
    words += align_up((tiles + 1) * sizeof(uint64_t)) / sizeof(uint32_t);
    m = tiles;
  }
  return words + 64;
}

template <typename T>
static int exclusive_scan(T *data, uint64_t n, T *scratch, hipStream_t s, CountOut co = CountOut{}) {
  if (n == 0) {
    // total of an empty array (a kernel, not a memset node, so the call can be captured)
    set_zero_kernel<T><<<1, 1, 0, s>>>(data, co);
    FGS_LAUNCH_CHECK("set_zero_kernel");
    return FGS_OK;
  }
  const uint64_t tiles = (n + kTile - 1) / kTile;
  if (tiles == 1) {
    scan_apply_kernel<T><<<1, kThreads, 0, s>>>(data, n, nullptr, 1, 0, co);
    FGS_LAUNCH_CHECK("scan_apply_kernel");
    return FGS_OK;
  }
  if (tiles > 0xffffffffull) return fail(FGS_E_UNSUPPORTED, "scan: too many elements");
  T *partial = scratch;
  T *rest = scratch + align_up((tiles + 1) * sizeof(T)) / sizeof(T);
  scan_reduce_kernel<T><<<unsigned(tiles), kThreads, 0, s>>>(data, n, partial);
  FGS_LAUNCH_CHECK("scan_reduce_kernel");
  // few tiles: each block adds up the sums before it (two launches in all);
  // many: the sums are scanned first
  const int self_prefix = tiles <= kSelfPrefixTiles ? 1 : 0;
  if (!self_prefix) {
    int st = exclusive_scan<T>(partial, tiles, rest, s);
    if (st != FGS_OK) return st;
  }
  scan_apply_kernel<T><<<unsigned(tiles), kThreads, 0, s>>>(data, n, partial, unsigned(tiles), self_prefix, co);
  FGS_LAUNCH_CHECK("scan_apply_kernel");
  return FGS_OK;
}

int exclusive_scan_u32(uint32_t *data, uint64_t n, uint32_t *scratch, hipStream_t s) {
  return exclusive_scan<uint32_t>(data, n, scratch, s);
}

int scan_counts(uint32_t *count, uint64_t n, uint32_t *scratch, uint64_t cap, unsigned long long *total,
                uint32_t *pairs, uint32_t *overflow, hipStream_t s) {
  return exclusive_scan<uint32_t>(count, n, scratch, s, CountOut{cap, total, pairs, overflow});
}

int exclusive_scan_u64(uint64_t *data, uint64_t n, uint32_t *scratch, hipStream_t s) {
  return exclusive_scan<uint64_t>(data, n, reinterpret_cast<uint64_t *>(scratch), s);
}

uint64_t sort_scratch_words(uint64_t n) {
  const uint64_t tiles = (n + kTile - 1) / kTile;
  const uint64_t table = uint64_t(kMaxBins) * tiles;
  return align_up((table + 1) * sizeof(uint32_t)) / sizeof(uint32_t) + scan_scratch_words(table);
}

int radix_sort_pairs(uint32_t *keys, uint32_t *vals, uint32_t *keys_alt, uint32_t *vals_alt,
                     uint64_t n, int bits, uint32_t *scratch, uint32_t **out_keys,
                     uint32_t **out_vals, hipStream_t s, int max_bits, const uint32_t *n_dev, int bit0) {
  *out_keys = keys;
  *out_vals = vals;
  if (n <= 1 || bits <= 0) return FGS_OK;
  if (n > 0xffffffffull) return fail(FGS_E_UNSUPPORTED, "sort: more than 2^32 pairs");
  const uint64_t tiles = (n + kTile - 1) / kTile;
  if (max_bits < 1 || max_bits > kSortMaxBits) return fail(FGS_E_INVALID, "sort: digit width");
  if (bit0 < 0 || bit0 + bits > 32) return fail(FGS_E_INVALID, "sort: key field outside 32 bits");
  const bool with_vals = vals != nullptr;
  const int passes = sort_passes(n, bits, max_bits);
  const int per = (bits + passes - 1) / passes;
  uint32_t *table = scratch;
  uint32_t *scan_tmp = scratch + align_up((uint64_t(kMaxBins) * tiles + 1) * sizeof(uint32_t)) / sizeof(uint32_t);
  uint32_t *ki = keys, *vi = vals, *ko = keys_alt, *vo = vals_alt;
  for (int p = 0, done = 0; p < passes; ++p, done += per) {
    const int nb = (bits - done < per) ? (bits - done) : per;
    const int shift = bit0 + done;
    const uint32_t mask = (1u << nb) - 1u;
    if (nb > 9)
      rs_hist_kernel<10><<<unsigned(tiles), kThreads, 0, s>>>(ki, n, n_dev, shift, mask, table, unsigned(tiles));
    else if (nb > 6)
      rs_hist_kernel<9><<<unsigned(tiles), kThreads, 0, s>>>(ki, n, n_dev, shift, mask, table, unsigned(tiles));
    else
      rs_hist_kernel<6><<<unsigned(tiles), kThreads, 0, s>>>(ki, n, n_dev, shift, mask, table, unsigned(tiles));
    FGS_LAUNCH_CHECK("rs_hist_kernel");
    int st = exclusive_scan_u32(table, uint64_t(mask + 1) * tiles, scan_tmp, s);
    if (st != FGS_OK) return st;
    auto scatter = [&](auto nbc, auto wv) {
      rs_scatter_kernel<decltype(nbc)::value, decltype(wv)::value><<<unsigned(tiles), kThreads, 0, s>>>(
          ki, vi, n, n_dev, shift, nb, table, unsigned(tiles), ko, vo);
    };
    using B10 = std::integral_constant<int, 10>;
    using B9 = std::integral_constant<int, 9>;
    using B6 = std::integral_constant<int, 6>;
    if (with_vals) {
      if (nb > 9) scatter(B10(), std::true_type()); else if (nb > 6) scatter(B9(), std::true_type());
      else scatter(B6(), std::true_type());
    } else {
      if (nb > 9) scatter(B10(), std::false_type()); else if (nb > 6) scatter(B9(), std::false_type());
      else scatter(B6(), std::false_type());
    }
    FGS_LAUNCH_CHECK("rs_scatter_kernel");
    uint32_t *t;
    t = ki; ki = ko; ko = t;
    t = vi; vi = vo; vo = t;
  }
  *out_keys = ki;
  *out_vals = vi;
  return FGS_OK;
}

}  // namespace fgs

namespace fgs {
namespace {

__global__ __launch_bounds__(256) void sum_chunks_kernel(const float *__restrict__ part, int chunks, uint64_t n,
                                                         float *__restrict__ out) {
  const uint64_t i = uint64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (i >= n) return;
  float acc = part[i];
  // eight loads in flight at a time, added in chunk order
  for (int c = 1; c < chunks; c += 8) {
    float x[8];
#pragma unroll
    for (int j = 0; j < 8; ++j) x[j] = c + j < chunks ? part[uint64_t(c + j) * n + i] : 0.f;
#pragma unroll
    for (int j = 0; j < 8; ++j)
      if (c + j < chunks) acc += x[j];
  }
  out[i] = acc;
}

}  // namespace

int sum_chunks(const float *part, int chunks, uint64_t n, float *out, hipStream_t s) {
  if (n == 0) return FGS_OK;
  sum_chunks_kernel<<<grid_for(n, 256), 256, 0, s>>>(part, chunks, n, out);
  FGS_LAUNCH_CHECK("sum_chunks_kernel");
  return FGS_OK;
}

}  // namespace fgs
