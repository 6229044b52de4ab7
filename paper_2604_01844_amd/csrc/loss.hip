// Loss, metric and optimiser kernels of the reconstruction loop:
// the L1 and 3D total-variation terms of Eq. 5 with their gradients, PSNR,
// and Adam.
// Reductions are two-level with a fixed block count, so results do not
// depend on timing (no atomics).
#include <cmath>

#include <algorithm>

#include "fgs_internal.h"

namespace fgs {
namespace {

constexpr int kRedThreads = 256;
constexpr int kRedBlocks = kLossBlocks;

// partial[b] = sum over this block's grid-stride share of |img - gt|; grad
// written alongside.
__global__ __launch_bounds__(kRedThreads) void l1_kernel(const float *__restrict__ img,
                                                         const float *__restrict__ gt, uint64_t n,
                                                         float inv_p, float *__restrict__ grad,
                                                         float *__restrict__ partial) {
  __shared__ float sh[kRedThreads / 64];
  CompSum acc;
  for (uint64_t i = uint64_t(blockIdx.x) * kRedThreads + threadIdx.x; i < n;
       i += uint64_t(gridDim.x) * kRedThreads) {
    const float d = img[i] - gt[i];
    acc.add(fabsf(d));
    if (grad) grad[i] = (d > 0.f) ? inv_p : ((d < 0.f) ? -inv_p : 0.f);
  }
  const float t = block_sum_f32<kRedThreads>(acc.value(), sh);
  if (threadIdx.x == 0) partial[blockIdx.x] = t;
}

__global__ __launch_bounds__(kRedThreads) void sq_err_kernel(const float *__restrict__ a,
                                                             const float *__restrict__ b, uint64_t n,
                                                             float *__restrict__ partial) {
  __shared__ float sh[kRedThreads / 64];
  CompSum acc;
  for (uint64_t i = uint64_t(blockIdx.x) * kRedThreads + threadIdx.x; i < n;
       i += uint64_t(gridDim.x) * kRedThreads) {
    const float d = a[i] - b[i];
    acc.add(d * d);
  }
  const float t = block_sum_f32<kRedThreads>(acc.value(), sh);
  if (threadIdx.x == 0) partial[blockIdx.x] = t;
}

// mode 0: out = scale * sum; mode 1: out = 10 log10(peak^2 / (sum / n)),
// with peak2_n = peak^2 * n formed on the host.
__global__ __launch_bounds__(kRedThreads) void finish_kernel(const float *__restrict__ partial, int nb,
                                                             int mode, float scale, float peak2_n,
                                                             float *__restrict__ out) {
  __shared__ float sh[kRedThreads / 64];
  CompSum acc;
  for (int i = threadIdx.x; i < nb; i += kRedThreads) acc.add(partial[i]);
  const float t = block_sum_f32<kRedThreads>(acc.value(), sh);
  if (threadIdx.x == 0) out[0] = (mode == 0) ? t * scale : 10.f * log10f(peak2_n / t);
}

__global__ __launch_bounds__(256) void adam_kernel(float *__restrict__ p, const float *__restrict__ g,
                                                   const float *__restrict__ g2,
                                                   float *__restrict__ m, float *__restrict__ v,
                                                   uint64_t n, float lr, float b1, float b2, float eps,
                                                   float c1, float c2, int clamp0) {
  const uint64_t i = uint64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const float gi = g2 ? g[i] + g2[i] : g[i];
  const float mi = b1 * m[i] + (1.f - b1) * gi;
  const float vi = b2 * v[i] + (1.f - b2) * gi * gi;
  m[i] = mi;
  v[i] = vi;
  const float mh = mi / c1;
  const float vh = vi / c2;
  float x = p[i] - lr * mh / (sqrtf(vh) + eps);
  if (clamp0) x = fmaxf(x, 0.f);
  p[i] = x;
}

// 3D total variation (the homogeneity prior of Eq. 5 on a sampled
// sub-volume): TV = (1/n) sum over voxels and axes of |V(i + e_a) - V(i)|
// (forward differences inside the grid), and its gradient
// dTV/dV(i) = (1/n) sum_a [sign(V(i) - V(i - e_a)) - sign(V(i + e_a) - V(i))],
// sign(0) = 0. Both scaled by `scale` (the loss weight). One thread per voxel.
__device__ __forceinline__ float sgn(float d) { return (d > 0.f) ? 1.f : ((d < 0.f) ? -1.f : 0.f); }

__global__ __launch_bounds__(kRedThreads) void tv_kernel(const float *__restrict__ vol, int nx, int ny, int nz,
                                                         float scale_n, float *__restrict__ grad,
                                                         float *__restrict__ partial) {
  __shared__ float sh[kRedThreads / 64];
  const uint64_t n = uint64_t(nx) * ny * nz;
  const uint64_t sy = uint64_t(nx), sz = uint64_t(nx) * ny;
  CompSum acc;
  for (uint64_t i = uint64_t(blockIdx.x) * kRedThreads + threadIdx.x; i < n;
       i += uint64_t(gridDim.x) * kRedThreads) {
    const int x = int(i % sy), y = int((i / sy) % ny), z = int(i / sz);
    const float v = vol[i];
    float g = 0.f;
    if (x + 1 < nx) { const float d = vol[i + 1] - v; acc.add(fabsf(d)); g -= sgn(d); }
    if (y + 1 < ny) { const float d = vol[i + sy] - v; acc.add(fabsf(d)); g -= sgn(d); }
    if (z + 1 < nz) { const float d = vol[i + sz] - v; acc.add(fabsf(d)); g -= sgn(d); }
    if (x > 0) g += sgn(v - vol[i - 1]);
    if (y > 0) g += sgn(v - vol[i - sy]);
    if (z > 0) g += sgn(v - vol[i - sz]);
    if (grad) grad[i] = g * scale_n;
  }
  const float t = block_sum_f32<kRedThreads>(acc.value(), sh);
  if (threadIdx.x == 0) partial[blockIdx.x] = t;
}

int reduce_blocks(uint64_t n) {
  uint64_t b = (n + kRedThreads - 1) / kRedThreads;
  return int(b < kRedBlocks ? (b ? b : 1) : kRedBlocks);
}

// The L1 term's two launches, with `partial` (at least reduce_blocks(n)
// floats of device memory) holding the per-block sums between them.
int launch_l1(const float *img, const float *gt, int64_t n_per_view, int32_t n_views, float *loss, float *grad,
              float *partial, hipStream_t s) {
  const uint64_t n = uint64_t(n_per_view) * uint64_t(n_views);
  const int nb = reduce_blocks(n);
  const float inv_p = 1.f / float(n_per_view);
  l1_kernel<<<nb, kRedThreads, 0, s>>>(img, gt, n, inv_p, grad, partial);
  FGS_LAUNCH_CHECK("l1_kernel");
  finish_kernel<<<1, kRedThreads, 0, s>>>(partial, nb, 0, float(1.0 / double(n_per_view)), 0.f, loss);
  FGS_LAUNCH_CHECK("finish_kernel");
  return FGS_OK;
}

}  // namespace

int loss_blocks(uint64_t n) { return reduce_blocks(n); }

int l1_partials(const float *img, const float *gt, uint64_t n, float inv_p, float *grad, float *partial,
                hipStream_t s) {
  l1_kernel<<<reduce_blocks(n), kRedThreads, 0, s>>>(img, gt, n, inv_p, grad, partial);
  FGS_LAUNCH_CHECK("l1_kernel");
  return FGS_OK;
}

int tv_partials(const float *vol, const int32_t dims[3], float scale, float *grad, float *partial,
                hipStream_t s) {
  const uint64_t n = uint64_t(dims[0]) * dims[1] * dims[2];
  tv_kernel<<<reduce_blocks(n), kRedThreads, 0, s>>>(vol, dims[0], dims[1], dims[2],
                                                     float(double(scale) / double(n)), grad, partial);
  FGS_LAUNCH_CHECK("tv_kernel");
  return FGS_OK;
}

}  // namespace fgs

using namespace fgs;

extern "C" int fgs_l1_loss_grad(const float *img, const float *gt, int64_t n_per_view, int32_t n_views,
                                float *loss, float *grad, fgs_workspace *ws, void *stream) {
  if (!img || !gt || !loss || !ws || !ws->ptr) return fail(FGS_E_INVALID, "null argument");
  if (n_per_view <= 0 || n_views <= 0) return fail(FGS_E_INVALID, "sizes");
  ws->needed = kRedBlocks * sizeof(float);
  if (ws->bytes < ws->needed) return fail(FGS_E_CAPACITY, "workspace too small");
  return launch_l1(img, gt, n_per_view, n_views, loss, grad, static_cast<float *>(ws->ptr),
                   static_cast<hipStream_t>(stream));
}

extern "C" int fgs_psnr(const float *vol, const float *ref, int64_t n, float peak, float *out,
                        fgs_workspace *ws, void *stream) {
  if (!vol || !ref || !out || !ws || !ws->ptr) return fail(FGS_E_INVALID, "null argument");
  if (n <= 0 || !(peak > 0.f)) return fail(FGS_E_INVALID, "sizes or peak");
  ws->needed = kRedBlocks * sizeof(float);
  if (ws->bytes < ws->needed) return fail(FGS_E_CAPACITY, "workspace too small");
  hipStream_t s = static_cast<hipStream_t>(stream);
  const int nb = reduce_blocks(uint64_t(n));
  float *partial = static_cast<float *>(ws->ptr);
  sq_err_kernel<<<nb, kRedThreads, 0, s>>>(vol, ref, uint64_t(n), partial);
  FGS_LAUNCH_CHECK("sq_err_kernel");
  finish_kernel<<<1, kRedThreads, 0, s>>>(partial, nb, 1, 0.f, float(double(peak) * double(peak) * double(n)),
                                          out);
  FGS_LAUNCH_CHECK("finish_kernel");
  return FGS_OK;
}

extern "C" int fgs_adam_step(float *param, const float *grad, const float *grad2, float *m, float *v,
                             int64_t n, int32_t step, float lr, float beta1, float beta2, float eps,
                             int32_t clamp_min_zero, void *stream) {
  if (!param || !grad || !m || !v) return fail(FGS_E_INVALID, "null argument");
  if (n <= 0 || step < 1) return fail(FGS_E_INVALID, "sizes or step");
  hipStream_t s = static_cast<hipStream_t>(stream);
  const float c1 = float(1.0 - std::pow(double(beta1), double(step)));
  const float c2 = float(1.0 - std::pow(double(beta2), double(step)));
  adam_kernel<<<grid_for(uint64_t(n), 256), 256, 0, s>>>(param, grad, grad2, m, v, uint64_t(n), lr, beta1, beta2, eps,
                                                         c1, c2, clamp_min_zero);
  FGS_LAUNCH_CHECK("adam_kernel");
  return FGS_OK;
}

namespace fgs {
namespace {

// Plain streaming copy, 16 bytes per thread per step (the reference kernel for
// HBM traffic counters: it reads and writes exactly 4 n bytes).
__global__ __launch_bounds__(256) void copy_kernel(const float4 *__restrict__ src, float4 *__restrict__ dst,
                                                   uint64_t n4) {
  for (uint64_t i = uint64_t(blockIdx.x) * blockDim.x + threadIdx.x; i < n4; i += uint64_t(gridDim.x) * blockDim.x)
    dst[i] = src[i];
}

}  // namespace
}  // namespace fgs

extern "C" int fgs_copy(const float *src, float *dst, int64_t n, void *stream) {
  if (!src || !dst || n < 0 || (n & 3) || (reinterpret_cast<uintptr_t>(src) & 15) ||
      (reinterpret_cast<uintptr_t>(dst) & 15))
    return fail(FGS_E_INVALID, "copy: 16-byte aligned buffers, n a multiple of 4");
  if (n == 0) return FGS_OK;
  hipStream_t s = static_cast<hipStream_t>(stream);
  const uint64_t n4 = uint64_t(n) / 4;
  const unsigned blocks = unsigned(std::min<uint64_t>((n4 + 255) / 256, 256u * 64u));
  copy_kernel<<<blocks, 256, 0, s>>>(reinterpret_cast<const float4 *>(src), reinterpret_cast<float4 *>(dst), n4);
  FGS_LAUNCH_CHECK("copy_kernel");
  return FGS_OK;
}

extern "C" int fgs_tv_loss_grad(const float *vol, const int32_t dims[3], float scale, float *loss, float *grad,
                                fgs_workspace *ws, void *stream) {
  if (!vol || !dims || !loss || !ws) return fail(FGS_E_INVALID, "null argument");
  if (dims[0] <= 0 || dims[1] <= 0 || dims[2] <= 0) return fail(FGS_E_INVALID, "dims must be >= 1");
  const uint64_t n = uint64_t(dims[0]) * dims[1] * dims[2];
  const int nb = reduce_blocks(n);
  ws->needed = uint64_t(nb) * sizeof(float);
  if (!ws->ptr || ws->bytes < ws->needed) return fail(FGS_E_CAPACITY, "workspace too small");
  ws->kind = 0;
  hipStream_t s = static_cast<hipStream_t>(stream);
  float *partial = static_cast<float *>(ws->ptr);
  tv_kernel<<<nb, kRedThreads, 0, s>>>(vol, dims[0], dims[1], dims[2], float(double(scale) / double(n)), grad,
                                       partial);
  FGS_LAUNCH_CHECK("tv_kernel");
  finish_kernel<<<1, kRedThreads, 0, s>>>(partial, nb, 0, float(double(scale) / double(n)), 0.f, loss);
  FGS_LAUNCH_CHECK("finish_kernel");
  return FGS_OK;
}
