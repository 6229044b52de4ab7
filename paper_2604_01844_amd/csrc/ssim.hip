// SSIM term of Eq. 5 (structural similarity between rendered and measured
// projections), fused: loss = scale * (1 - mean SSIM) and its gradient with
// respect to the rendered image.
//
// Local statistics use the 11-tap Gaussian window (sigma 1.5) with zero
// padding: mx, my, E[x^2], E[y^2], E[xy]. With
//   A = 2 mx my + c1, B = 2 (E[xy] - mx my) + c2,
//   C = mx^2 + my^2 + c1, D = E[x^2] - mx^2 + E[y^2] - my^2 + c2,
// SSIM = A B / (C D), and, per pixel p,
//   d(mean SSIM)/dx(p) = (1/n) [ (w * G1)(p) + 2 x(p) (w * G2)(p) + y(p) (w * G3)(p) ]
// where G1, G2, G3 are dSSIM/d(mx, E[x^2], E[xy]) (the window is symmetric,
// so the adjoint of the windowed sum is the windowed sum).
//
// Two kernels over 32x32 output tiles with a 5-pixel halo staged in LDS,
// each a separable (horizontal then vertical) 11-tap pass:
//   stats kernel: the five statistics, 1 - SSIM (block partial sums, no atomics)
//                 and the three G maps;
//   grad kernel:  the windowed sums of the G maps and the gradient.
// The 3D variant (the fitting loss of Eq. 6) is at the end of the file.
#include <algorithm>
#include <cmath>

#include "fgs_internal.h"

namespace fgs {
namespace {

constexpr int kR = 5;              // window radius
constexpr int kWin = 2 * kR + 1;   // 11 taps
constexpr int kT = 32;             // output tile side
constexpr int kH = kT + 2 * kR;    // staged side (42)
constexpr int kThreads = 256;

struct Window {
  float w[kWin];
};

// Normalised 11-tap Gaussian window, sigma 1.5 (computed in double).
Window gaussian_window() {
  Window win;
  double wsum = 0.0, wd[kWin];
  for (int k = 0; k < kWin; ++k) {
    const double d = double(k - kR);
    wd[k] = std::exp(-d * d / (2.0 * 1.5 * 1.5));
    wsum += wd[k];
  }
  for (int k = 0; k < kWin; ++k) win.w[k] = float(wd[k] / wsum);
  return win;
}

__global__ __launch_bounds__(kThreads) void ssim_stats_kernel(const float *__restrict__ img,
                                                              const float *__restrict__ gt, int W, int H,
                                                              Window win, float c1, float c2,
                                                              float *__restrict__ g1, float *__restrict__ g2,
                                                              float *__restrict__ g3,
                                                              float *__restrict__ partial) {
  __shared__ float sx[kH][kH + 1], sy[kH][kH + 1];
  __shared__ float hz[5][kH][kT + 1];
  __shared__ float sh[kThreads / 64];
  const int x0 = blockIdx.x * kT, y0 = blockIdx.y * kT, v = blockIdx.z;
  const uint64_t off = uint64_t(v) * uint64_t(W) * uint64_t(H);
  for (int i = threadIdx.x; i < kH * kH; i += kThreads) {
    const int r = i / kH, c = i - r * kH;
    const int gx = x0 - kR + c, gy = y0 - kR + r;
    const bool in = gx >= 0 && gx < W && gy >= 0 && gy < H;
    const uint64_t q = off + uint64_t(gy) * W + gx;
    sx[r][c] = in ? img[q] : 0.f;
    sy[r][c] = in ? gt[q] : 0.f;
  }
  __syncthreads();
  for (int i = threadIdx.x; i < kH * kT; i += kThreads) {
    const int r = i / kT, c = i - r * kT;
    float a = 0.f, b = 0.f, aa = 0.f, bb = 0.f, ab = 0.f;
#pragma unroll
    for (int k = 0; k < kWin; ++k) {
      const float xv = sx[r][c + k], yv = sy[r][c + k], wk = win.w[k];
      a = fmaf(wk, xv, a);
      b = fmaf(wk, yv, b);
      aa = fmaf(wk * xv, xv, aa);
      bb = fmaf(wk * yv, yv, bb);
      ab = fmaf(wk * xv, yv, ab);
    }
    hz[0][r][c] = a; hz[1][r][c] = b; hz[2][r][c] = aa; hz[3][r][c] = bb; hz[4][r][c] = ab;
  }
  __syncthreads();
  CompSum acc;
  for (int i = threadIdx.x; i < kT * kT; i += kThreads) {
    const int r = i / kT, c = i - r * kT;
    float m[5] = {0.f, 0.f, 0.f, 0.f, 0.f};
#pragma unroll
    for (int k = 0; k < kWin; ++k)
#pragma unroll
      for (int j = 0; j < 5; ++j) m[j] = fmaf(win.w[k], hz[j][r + k][c], m[j]);
    const int gx = x0 + c, gy = y0 + r;
    if (gx >= W || gy >= H) continue;
    const float mx = m[0], my = m[1];
    const float A = fmaf(2.f * mx, my, c1);
    const float B = fmaf(2.f, m[4] - mx * my, c2);
    const float C = fmaf(mx, mx, fmaf(my, my, c1));
    const float D = (m[2] - mx * mx) + (m[3] - my * my) + c2;
    const float CD = C * D;
    const float S = A * B / CD;
    acc.add(1.f - S);
    const uint64_t q = off + uint64_t(gy) * W + gx;
    if (g1) {
      g1[q] = 2.f * my * (B - A) / CD - S * (2.f * mx / C - 2.f * mx / D);
      g2[q] = -S / D;
      g3[q] = 2.f * A / CD;
    }
  }
  const float t = block_sum_f32<kThreads>(acc.value(), sh);
  if (threadIdx.x == 0)
    partial[(uint64_t(blockIdx.z) * gridDim.y + blockIdx.y) * gridDim.x + blockIdx.x] = t;
}

__global__ __launch_bounds__(kThreads) void ssim_grad_kernel(const float *__restrict__ img,
                                                             const float *__restrict__ gt, int W, int H,
                                                             Window win, const float *__restrict__ g1,
                                                             const float *__restrict__ g2,
                                                             const float *__restrict__ g3, float coef,
                                                             int accumulate, float *__restrict__ grad) {
  __shared__ float sg[3][kH][kH + 1];
  __shared__ float hz[3][kH][kT + 1];
  const int x0 = blockIdx.x * kT, y0 = blockIdx.y * kT, v = blockIdx.z;
  const uint64_t off = uint64_t(v) * uint64_t(W) * uint64_t(H);
  for (int i = threadIdx.x; i < kH * kH; i += kThreads) {
    const int r = i / kH, c = i - r * kH;
    const int gx = x0 - kR + c, gy = y0 - kR + r;
    const bool in = gx >= 0 && gx < W && gy >= 0 && gy < H;
    const uint64_t q = off + uint64_t(gy) * W + gx;
    sg[0][r][c] = in ? g1[q] : 0.f;
    sg[1][r][c] = in ? g2[q] : 0.f;
    sg[2][r][c] = in ? g3[q] : 0.f;
  }
  __syncthreads();
  for (int i = threadIdx.x; i < kH * kT; i += kThreads) {
    const int r = i / kT, c = i - r * kT;
    float a[3] = {0.f, 0.f, 0.f};
#pragma unroll
    for (int k = 0; k < kWin; ++k)
#pragma unroll
      for (int j = 0; j < 3; ++j) a[j] = fmaf(win.w[k], sg[j][r][c + k], a[j]);
#pragma unroll
    for (int j = 0; j < 3; ++j) hz[j][r][c] = a[j];
  }
  __syncthreads();
  for (int i = threadIdx.x; i < kT * kT; i += kThreads) {
    const int r = i / kT, c = i - r * kT;
    const int gx = x0 + c, gy = y0 + r;
    if (gx >= W || gy >= H) continue;
    float a[3] = {0.f, 0.f, 0.f};
#pragma unroll
    for (int k = 0; k < kWin; ++k)
#pragma unroll
      for (int j = 0; j < 3; ++j) a[j] = fmaf(win.w[k], hz[j][r + k][c], a[j]);
    const uint64_t q = off + uint64_t(gy) * W + gx;
    const float gq = coef * (a[0] + 2.f * img[q] * a[1] + gt[q] * a[2]);
    grad[q] = accumulate ? grad[q] + gq : gq;
  }
}

// The partial sums are of 1 - SSIM (no cancellation when SSIM is near 1):
// loss = (scale / n) * their total.
__global__ __launch_bounds__(kThreads) void ssim_finish_kernel(const float *__restrict__ partial, int nb,
                                                               float scale_n, float *__restrict__ loss) {
  __shared__ float sh[kThreads / 64];
  CompSum acc;
  for (int i = threadIdx.x; i < nb; i += kThreads) acc.add(partial[i]);
  const float t = block_sum_f32<kThreads>(acc.value(), sh);
  if (threadIdx.x == 0) loss[0] = scale_n * t;
}

}  // namespace
}  // namespace fgs

using namespace fgs;

extern "C" int fgs_ssim_loss_grad(const float *img, const float *gt, int32_t W, int32_t H, int32_t n_views,
                                  float c1, float c2, float scale, float *loss, float *grad,
                                  int32_t accumulate, fgs_workspace *ws, void *stream) {
  if (!img || !gt || !loss || !ws) return fail(FGS_E_INVALID, "null argument");
  if (W <= 0 || H <= 0 || n_views <= 0 || n_views > 65535) return fail(FGS_E_INVALID, "image sizes");
  if (!(c1 > 0.f) || !(c2 > 0.f)) return fail(FGS_E_INVALID, "c1 and c2 must be > 0");
  const uint64_t n = uint64_t(W) * uint64_t(H) * uint64_t(n_views);
  const dim3 grid(unsigned((W + kT - 1) / kT), unsigned((H + kT - 1) / kT), unsigned(n_views));
  const uint64_t nb = uint64_t(grid.x) * grid.y * grid.z;
  Carver c(nullptr);
  uint64_t o_part, o_g;
  c.take<float>(nb, &o_part);
  c.take<float>(grad ? 3 * n : 0, &o_g);
  ws->needed = c.used;
  if (!ws->ptr || ws->bytes < ws->needed) return fail(FGS_E_CAPACITY, "workspace too small");
  ws->kind = 0;
  char *b = static_cast<char *>(ws->ptr);
  float *partial = reinterpret_cast<float *>(b + o_part);
  float *g1 = grad ? reinterpret_cast<float *>(b + o_g) : nullptr;
  float *g2 = grad ? g1 + n : nullptr;
  float *g3 = grad ? g2 + n : nullptr;
  const Window win = gaussian_window();
  hipStream_t s = static_cast<hipStream_t>(stream);
  ssim_stats_kernel<<<grid, kThreads, 0, s>>>(img, gt, W, H, win, c1, c2, g1, g2, g3, partial);
  FGS_LAUNCH_CHECK("ssim_stats_kernel");
  ssim_finish_kernel<<<1, kThreads, 0, s>>>(partial, int(nb), float(double(scale) / double(n)), loss);
  FGS_LAUNCH_CHECK("ssim_finish_kernel");
  if (grad) {
    ssim_grad_kernel<<<grid, kThreads, 0, s>>>(img, gt, W, H, win, g1, g2, g3, float(-double(scale) / double(n)),
                                               accumulate, grad);
    FGS_LAUNCH_CHECK("ssim_grad_kernel");
  }
  return FGS_OK;
}

// ---------------------------------------------------------------------------
// 3D SSIM (the fitting loss of Eq. 6): the same per-voxel formula with the
// separable 11^3 window, as three 1D passes (x, then y, then z) over
// channel-major volumes, one thread per output voxel and all channels; no
// atomics (block partial sums for the mean).

namespace fgs {
namespace {

// out[c][i] = sum_k w[k] in_c(i + (k - 5) e_axis), zero outside the grid.
// first pass (products != 0): the 5 channels are formed from x and y:
// x, y, x^2, y^2, x y.
template <int CH, bool PRODUCTS>
__global__ __launch_bounds__(256) void sep_pass_kernel(const float *__restrict__ in, const float *__restrict__ y_in,
                                                       int nx, int ny, int nz, int axis, Window win,
                                                       float *__restrict__ out) {
  const uint64_t n = uint64_t(nx) * ny * nz;
  const uint64_t i = uint64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const int x = int(i % uint64_t(nx));
  const int yy = int((i / uint64_t(nx)) % uint64_t(ny));
  const int z = int(i / (uint64_t(nx) * ny));
  const int pos = axis == 0 ? x : (axis == 1 ? yy : z);
  const int len = axis == 0 ? nx : (axis == 1 ? ny : nz);
  const int64_t stride = axis == 0 ? 1 : (axis == 1 ? int64_t(nx) : int64_t(nx) * ny);
  float acc[CH];
#pragma unroll
  for (int c = 0; c < CH; ++c) acc[c] = 0.f;
#pragma unroll
  for (int k = 0; k < kWin; ++k) {
    const int p = pos + k - kR;
    if (p < 0 || p >= len) continue;
    const uint64_t j = uint64_t(int64_t(i) + int64_t(k - kR) * stride);
    const float wk = win.w[k];
    if (PRODUCTS) {
      const float xv = in[j], yv = y_in[j];
      acc[0] = fmaf(wk, xv, acc[0]);
      acc[1] = fmaf(wk, yv, acc[1]);
      acc[2] = fmaf(wk * xv, xv, acc[2]);
      acc[3] = fmaf(wk * yv, yv, acc[3]);
      acc[4] = fmaf(wk * xv, yv, acc[4]);
    } else {
#pragma unroll
      for (int c = 0; c < CH; ++c) acc[c] = fmaf(wk, in[uint64_t(c) * n + j], acc[c]);
    }
  }
#pragma unroll
  for (int c = 0; c < CH; ++c) out[uint64_t(c) * n + i] = acc[c];
}

// From the windowed statistics m[5][n]: SSIM partial sums and G maps g[3][n].
__global__ __launch_bounds__(256) void ssim_map_kernel(const float *__restrict__ m, uint64_t n, float c1, float c2,
                                                       float *__restrict__ g, float *__restrict__ partial) {
  __shared__ float sh[kThreads / 64];
  CompSum acc;
  for (uint64_t i = uint64_t(blockIdx.x) * kThreads + threadIdx.x; i < n; i += uint64_t(gridDim.x) * kThreads) {
    const float mx = m[i], my = m[n + i];
    const float A = fmaf(2.f * mx, my, c1);
    const float B = fmaf(2.f, m[4 * n + i] - mx * my, c2);
    const float C = fmaf(mx, mx, fmaf(my, my, c1));
    const float D = (m[2 * n + i] - mx * mx) + (m[3 * n + i] - my * my) + c2;
    const float CD = C * D;
    const float S = A * B / CD;
    acc.add(1.f - S);
    if (g) {
      g[i] = 2.f * my * (B - A) / CD - S * (2.f * mx / C - 2.f * mx / D);
      g[n + i] = -S / D;
      g[2 * n + i] = 2.f * A / CD;
    }
  }
  const float t = block_sum_f32<kThreads>(acc.value(), sh);
  if (threadIdx.x == 0) partial[blockIdx.x] = t;
}

__global__ __launch_bounds__(256) void ssim_combine_kernel(const float *__restrict__ vol, const float *__restrict__ gt,
                                                           const float *__restrict__ cg, uint64_t n, float coef,
                                                           int accumulate, float *__restrict__ grad) {
  const uint64_t i = uint64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const float gq = coef * (cg[i] + 2.f * vol[i] * cg[n + i] + gt[i] * cg[2 * n + i]);
  grad[i] = accumulate ? grad[i] + gq : gq;
}

}  // namespace
}  // namespace fgs

extern "C" int fgs_ssim3d_loss_grad(const float *vol, const float *gt, const int32_t dims[3], float c1, float c2,
                                    float scale, float *loss, float *grad, int32_t accumulate, fgs_workspace *ws,
                                    void *stream) {
  if (!vol || !gt || !dims || !loss || !ws) return fail(FGS_E_INVALID, "null argument");
  if (dims[0] <= 0 || dims[1] <= 0 || dims[2] <= 0) return fail(FGS_E_INVALID, "dims must be >= 1");
  if (!(c1 > 0.f) || !(c2 > 0.f)) return fail(FGS_E_INVALID, "c1 and c2 must be > 0");
  const int nx = dims[0], ny = dims[1], nz = dims[2];
  const uint64_t n = uint64_t(nx) * ny * nz;
  const int nb = int(std::min<uint64_t>((n + kThreads - 1) / kThreads, 1024));
  Carver c(nullptr);
  uint64_t o_a, o_b, o_part;
  c.take<float>(5 * n, &o_a);
  c.take<float>(5 * n, &o_b);
  c.take<float>(uint64_t(nb), &o_part);
  ws->needed = c.used;
  if (!ws->ptr || ws->bytes < ws->needed) return fail(FGS_E_CAPACITY, "workspace too small");
  ws->kind = 0;
  char *b = static_cast<char *>(ws->ptr);
  float *ba = reinterpret_cast<float *>(b + o_a), *bb = reinterpret_cast<float *>(b + o_b);
  float *partial = reinterpret_cast<float *>(b + o_part);
  const Window win = gaussian_window();
  hipStream_t s = static_cast<hipStream_t>(stream);
  const unsigned g1 = grid_for(n, 256);
  sep_pass_kernel<5, true><<<g1, 256, 0, s>>>(vol, gt, nx, ny, nz, 0, win, ba);
  sep_pass_kernel<5, false><<<g1, 256, 0, s>>>(ba, nullptr, nx, ny, nz, 1, win, bb);
  sep_pass_kernel<5, false><<<g1, 256, 0, s>>>(bb, nullptr, nx, ny, nz, 2, win, ba);
  FGS_LAUNCH_CHECK("sep_pass_kernel");
  ssim_map_kernel<<<nb, kThreads, 0, s>>>(ba, n, c1, c2, grad ? bb : nullptr, partial);
  FGS_LAUNCH_CHECK("ssim_map_kernel");
  ssim_finish_kernel<<<1, kThreads, 0, s>>>(partial, nb, float(double(scale) / double(n)), loss);
  FGS_LAUNCH_CHECK("ssim_finish_kernel");
  if (grad) {
    sep_pass_kernel<3, false><<<g1, 256, 0, s>>>(bb, nullptr, nx, ny, nz, 0, win, ba);
    sep_pass_kernel<3, false><<<g1, 256, 0, s>>>(ba, nullptr, nx, ny, nz, 1, win, bb);
    sep_pass_kernel<3, false><<<g1, 256, 0, s>>>(bb, nullptr, nx, ny, nz, 2, win, ba);
    FGS_LAUNCH_CHECK("sep_pass_kernel");
    ssim_combine_kernel<<<g1, 256, 0, s>>>(vol, gt, ba, n, float(-double(scale) / double(n)), accumulate, grad);
    FGS_LAUNCH_CHECK("ssim_combine_kernel");
  }
  return FGS_OK;
}
