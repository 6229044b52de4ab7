// Internal declarations of libfactgs: error reporting, workspace carving,
// launch helpers and the per-Gaussian device math shared by the rasterizer
// and voxelizer kernels. Not part of the public ABI (include/factgs.h).
#pragma once

#include <hip/hip_runtime.h>

#include <cstddef>
#include <cstdint>
#include <string>
#include <type_traits>

#include "factgs.h"

namespace fgs {

// Independent tiles (one per wave) per workgroup of the pixel and voxel
// kernels: 16 when a call has enough tiles to give every CU several
// workgroups (which is what lets a CU hold enough waves), fewer for small
// calls (one view, a crop) so that their waves spread over all CUs.
// A workgroup's LDS is released only when all its waves are done, so a wave
// that finishes its tile early leaves its slot idle until the workgroup's
// longest tile ends. small_blocks = true caps large calls at 4 tiles per
// workgroup: this pays where tile lists are long and uneven, and costs a
// little (more workgroups to dispatch) where they are short.
inline int tiles_per_block(uint64_t n_tiles, bool small_blocks = false) {
  return n_tiles >= 16384 ? (small_blocks ? 4 : 16) : (n_tiles >= 4096 ? 4 : 1);
}

// Waves per tile: a call with few tiles (one view, a crop) splits each
// tile's list over several waves (strided batches), so that the longest
// list does not set the kernel time; large calls keep one wave per tile.
inline int chunks_per_tile(uint64_t n_tiles) {
  if (n_tiles >= 8192) return 1;
  const uint64_t c = (8192 + n_tiles - 1) / n_tiles;
  return int(c < 16 ? c : 16);
}

// Key emission is block-cooperative: a block of kEmitBlock threads takes up
// to kEmitBlock consecutive records and writes their keys (which are
// contiguous after the scan) in coalesced rounds, each thread finding its
// key's record by binary search over the block's offsets in LDS.
constexpr int kEmitBlock = 256;

// Largest i in [0, n) with off[i] <= q, for off ascending (off[0] <= q).
__device__ __forceinline__ int upper_index(const uint32_t *off, int n, uint32_t q) {
  int lo = 0, hi = n - 1;
  while (lo < hi) {
    const int mid = (lo + hi + 1) >> 1;
    if (off[mid] <= q) lo = mid; else hi = mid - 1;
  }
  return lo;
}

// out[i] = sum over c = 0..chunks-1 (in order) of part[c * n + i].
int sum_chunks(const float *part, int chunks, uint64_t n, float *out, hipStream_t s);

// fgs_voxelize_fwd / fgs_voxelize_bwd with the grid origin (3 floats) read on
// the device from origin_dev when it is not null (grid->origin is then not
// read by the kernels): a step captured in a graph can move its crop between
// replays. The tile layout depends on grid->dims and spacing only.
int vox_forward(const fgs_gaussians *g, const fgs_grid *grid, const fgs_opts *opts, float *vol, fgs_workspace *ws,
                hipStream_t s, const float *origin_dev);
int vox_backward(const fgs_gaussians *g, const fgs_grid *grid, const fgs_opts *opts, const float *grad_vol,
                 fgs_gaussian_grads *out, fgs_workspace *ws, hipStream_t s, const float *origin_dev);

// XCD-aware block order. MI355X has 8 XCDs, each with its own L2, and hands
// out consecutive workgroups round-robin over them. Renumbering so that XCD x
// takes the x-th contiguous eighth of the blocks keeps neighbouring tiles,
// which read the same records, in one L2. A bijection of [0, n).
constexpr uint32_t kXcds = 8;
__device__ __forceinline__ uint32_t xcd_block(uint32_t b, uint32_t n) {
  const uint32_t x = b % kXcds, q = b / kXcds;
  const uint32_t base = n / kXcds, rem = n % kXcds;
  return x * base + (x < rem ? x : rem) + q;
}

// Calls f(std::integral_constant<int, TPB>) with TPB = tiles_per_block(n_tiles, small_blocks).
template <typename F>
void with_tiles_per_block(uint64_t n_tiles, F &&f, bool small_blocks = false) {
  switch (tiles_per_block(n_tiles, small_blocks)) {
    case 16: f(std::integral_constant<int, 16>()); break;
    case 4: f(std::integral_constant<int, 4>()); break;
    default: f(std::integral_constant<int, 1>()); break;
  }
}


// ------------------------------------------------------------------ errors

void set_error(const std::string &msg);
int fail(int code, const std::string &msg);
int hip_fail(hipError_t e, const char *what);

#define FGS_HIP(call)                                     \
  do {                                                    \
    hipError_t e_ = (call);                               \
    if (e_ != hipSuccess) return ::fgs::hip_fail(e_, #call); \
  } while (0)

#define FGS_LAUNCH_CHECK(what)                            \
  do {                                                    \
    hipError_t e_ = hipGetLastError();                    \
    if (e_ != hipSuccess) return ::fgs::hip_fail(e_, what); \
  } while (0)

// ------------------------------------------------------------- workspace

constexpr uint64_t kAlign = 256;

inline uint64_t align_up(uint64_t x) { return (x + kAlign - 1) / kAlign * kAlign; }

// Sequential carving of a caller-owned buffer. Offsets only; `base` may be
// null when the carver is used just to measure the total.
struct Carver {
  char *base;
  uint64_t used = 0;
  explicit Carver(void *b) : base(static_cast<char *>(b)) {}
  template <typename T>
  T *take(uint64_t count, uint64_t *offset_out = nullptr) {
    uint64_t off = used;
    used = align_up(used + count * sizeof(T));
    if (offset_out) *offset_out = off;
    return base ? reinterpret_cast<T *>(base + off) : nullptr;
  }
};

// ----------------------------------------------------------- scan / sort

// Exclusive prefix sum of n uint32 values, in place: data[n] receives the
// total. data must hold n + 1 entries. Scratch from scan_scratch_words(n).
// Scratch is counted in 32-bit words (8-byte aligned inside the workspace).
uint64_t scan_scratch_words(uint64_t n);
int exclusive_scan_u32(uint32_t *data, uint64_t n, uint32_t *scratch, hipStream_t s);
int exclusive_scan_u64(uint64_t *data, uint64_t n, uint32_t *scratch, hipStream_t s);

// Widest digit of one radix-sort pass (1024 bins).
constexpr int kSortMaxBits = 10;

// Passes radix_sort_pairs makes over n pairs sorted on `bits` bits with
// digits of at most max_bits; the result ends in the alternate buffers when
// this is odd.
inline int sort_passes(uint64_t n, int bits, int max_bits = kSortMaxBits) {
  return (n > 1 && bits > 0) ? (bits + max_bits - 1) / max_bits : 0;
}

// Stable LSD radix sort of (key, value) uint32 pairs on bits [bit0, bit0 +
// bits) of the key. Input in keys/vals; the sorted result ends in the
// buffers returned through out_keys/out_vals (either the inputs or the
// alternates). vals == nullptr: keys only (one word per item: half the
// bytes per pass; out_vals is then null). n_dev (may be null): a device
// word holding the number of pairs, at most n; the launches are sized for n
// and sort only that many (no host wait).
uint64_t sort_scratch_words(uint64_t n);
int radix_sort_pairs(uint32_t *keys, uint32_t *vals, uint32_t *keys_alt, uint32_t *vals_alt,
                     uint64_t n, int bits, uint32_t *scratch, uint32_t **out_keys,
                     uint32_t **out_vals, hipStream_t s, int max_bits = kSortMaxBits,
                     const uint32_t *n_dev = nullptr, int bit0 = 0);

// Exclusive scan of a binning's per-record key counts (n values, each
// tile of 4096 summing below 2^32; count[n] = the 32-bit total) that also
// gives its pair count without a host wait: *total = the 64-bit sum;
// pairs[0] = the sum if it is at most cap, else 0 (nothing is binned);
// pairs[1] = 1 if the sum exceeds cap, else 0. A non-null `overflow` (device
// uint32[2]) on an excess: overflow[0] = 1 and overflow[1] raised to the sum
// (clamped to 2^32 - 1). scratch: scan_scratch_words(n) words.
int scan_counts(uint32_t *count, uint64_t n, uint32_t *scratch, uint64_t cap, unsigned long long *total,
                uint32_t *pairs, uint32_t *overflow, hipStream_t s);

// Loss terms of the optimiser step that leave their per-block partial sums
// for one later reduction (the step adds them up in its Adam launch):
// loss_blocks(n): the partial sums of the L1 or TV term over n values (at
// most kLossBlocks); l1_partials: the L1 term of Eq. 5, grad = sign(img -
// gt) * inv_p; tv_partials: the crop TV term with its gradient (scale / n
// per sign); ssim_l1_partials: the SSIM term of one W x H view (partials
// per 16 x 16 tile, ssim_tiles of them) with, for l1_inv_p > 0, the L1 term
// fused in (its partials per tile too), grad = L1 + SSIM gradient written
// (not added); gmaps: 3 W H floats of scratch.
constexpr int kLossBlocks = 1024;
int loss_blocks(uint64_t n);
int l1_partials(const float *img, const float *gt, uint64_t n, float inv_p, float *grad, float *partial,
                hipStream_t s);
int tv_partials(const float *vol, const int32_t dims[3], float scale, float *grad, float *partial,
                hipStream_t s);
uint64_t ssim_tiles(int32_t W, int32_t H);
int ssim_l1_partials(const float *img, const float *gt, int32_t W, int32_t H, float c1, float c2, float scale,
                     float l1_inv_p, float *grad, float *gmaps, float *part_ssim, float *part_l1, hipStream_t s);

inline int bits_for(uint64_t n_values) {  // bits needed to hold 0 .. n_values - 1
  int b = 0;
  while ((uint64_t(1) << b) < n_values) ++b;
  return b;
}

inline unsigned grid_for(uint64_t n, unsigned block) {
  return static_cast<unsigned>((n + block - 1) / block);
}

// ------------------------------------------------------------ device math

// Orders one wavefront's LDS accesses: writes issued before are visible to
// reads issued after, by any lane of the same wave (LDS operations of a wave
// complete in order). Used where each wave of a workgroup owns its own tile
// and its own LDS slice, so no workgroup barrier is needed.
__device__ __forceinline__ void wave_lds_sync() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

// Compensated FP32 accumulation (Neumaier's form of Kahan summation): the
// running error term keeps a long sequential sum within a few ulps of its
// exact value. Scalar reductions (losses, metrics) accumulate each thread's
// strided share with it; lanes, waves and blocks are then combined by
// pairwise trees, so every result is FP32 and independent of timing.
struct CompSum {
  float s = 0.f, c = 0.f;
  __device__ __forceinline__ void add(float x) {
    const float t = s + x;
    c += (fabsf(s) >= fabsf(x)) ? ((s - t) + x) : ((x - t) + s);
    s = t;
  }
  __device__ __forceinline__ float value() const { return s + c; }
};

// Sum of v over a workgroup of NT threads (NT a multiple of 64): an xor
// butterfly inside each wave, then the wave totals pairwise. The result is
// valid in thread 0 only. sh holds NT / 64 floats. Contains a barrier: every
// thread of the workgroup must call it.
template <int NT>
__device__ __forceinline__ float block_sum_f32(float v, float *sh) {
  static_assert(NT % 64 == 0 && NT <= 1024, "workgroup of whole waves");
#pragma unroll
  for (int d = 32; d > 0; d >>= 1) v += __shfl_xor(v, d, 64);
  if ((threadIdx.x & 63) == 0) sh[threadIdx.x >> 6] = v;
  __syncthreads();
  float t = 0.f;
  if (threadIdx.x == 0) {
    float w[NT / 64];
#pragma unroll
    for (int i = 0; i < NT / 64; ++i) w[i] = sh[i];
#pragma unroll
    for (int step = 1; step < NT / 64; step *= 2)
#pragma unroll
      for (int i = 0; i + step < NT / 64; i += 2 * step) w[i] += w[i + step];
    t = w[0];
  }
  return t;
}

// log2(e): exp(x) = exp2(x * log2(e)). Kernels pre-scale quadratic forms by
// -log2(e)/2 so that the Gaussian factor is a single v_exp_f32.
constexpr float kLog2e = 1.4426950408889634f;
constexpr float kTwoPi = 6.283185307179586f;

struct Mat3 {
  float m[9];
};

// Rotation of the normalised quaternion q = (w, x, y, z), Hamilton convention.
__device__ __forceinline__ void quat_to_rot(float w, float x, float y, float z, float R[9]) {
  R[0] = 1.f - 2.f * (y * y + z * z);
  R[1] = 2.f * (x * y - w * z);
  R[2] = 2.f * (x * z + w * y);
  R[3] = 2.f * (x * y + w * z);
  R[4] = 1.f - 2.f * (x * x + z * z);
  R[5] = 2.f * (y * z - w * x);
  R[6] = 2.f * (x * z - w * y);
  R[7] = 2.f * (y * z + w * x);
  R[8] = 1.f - 2.f * (x * x + y * y);
}

// Chain rule through quat_to_rot and the normalisation q_hat = q / |q|:
// dq = (I - q_hat q_hat^T) dq_hat / |q|, dq_hat from dR.
__device__ __forceinline__ void rot_grad_to_quat(const float qh[4], float qnorm, const float dR[9],
                                                 float dq[4]) {
  const float w = qh[0], x = qh[1], y = qh[2], z = qh[3];
  float gw = 2.f * (-z * dR[1] + y * dR[2] + z * dR[3] - x * dR[5] - y * dR[6] + x * dR[7]);
  float gx = 2.f * (y * dR[1] + z * dR[2] + y * dR[3] - 2.f * x * dR[4] - w * dR[5] + z * dR[6] +
                    w * dR[7] - 2.f * x * dR[8]);
  float gy = 2.f * (-2.f * y * dR[0] + x * dR[1] + w * dR[2] + x * dR[3] + z * dR[5] - w * dR[6] +
                    z * dR[7] - 2.f * y * dR[8]);
  float gz = 2.f * (-2.f * z * dR[0] - w * dR[1] + x * dR[2] + w * dR[3] - 2.f * z * dR[4] +
                    y * dR[5] + x * dR[6] + y * dR[7]);
  float dot = gw * w + gx * x + gy * y + gz * z;
  float inv = 1.f / qnorm;
  dq[0] = (gw - w * dot) * inv;
  dq[1] = (gx - x * dot) * inv;
  dq[2] = (gy - y * dot) * inv;
  dq[3] = (gz - z * dot) * inv;
}

// One Gaussian's parameters as loaded from the SoA inputs.
struct GaussParams {
  float p[3];
  float s[3];    // standard deviations exp(log_scale)
  float qh[4];   // normalised quaternion
  float qnorm;
  float R[9];    // rotation (columns are principal axes)
  float rho;
};

__device__ __forceinline__ void load_gauss(const fgs_gaussians &g, int64_t i, GaussParams &G) {
  const int64_t n = g.n;
  G.p[0] = g.mean[i];
  G.p[1] = g.mean[n + i];
  G.p[2] = g.mean[2 * n + i];
  G.s[0] = expf(g.log_scale[i]);
  G.s[1] = expf(g.log_scale[n + i]);
  G.s[2] = expf(g.log_scale[2 * n + i]);
  float w = g.quat[i], x = g.quat[n + i], y = g.quat[2 * n + i], z = g.quat[3 * n + i];
  float nn = sqrtf(w * w + x * x + y * y + z * z);
  G.qnorm = nn;
  float inv = 1.f / nn;
  G.qh[0] = w * inv;
  G.qh[1] = x * inv;
  G.qh[2] = y * inv;
  G.qh[3] = z * inv;
  quat_to_rot(G.qh[0], G.qh[1], G.qh[2], G.qh[3], G.R);
  G.rho = g.density[i];
}

}  // namespace fgs
