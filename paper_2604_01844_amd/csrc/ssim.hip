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
//   stats kernel: the five statistics, SSIM (block partial sums, no atomics)
//                 and the three G maps;
//   grad kernel:  the windowed sums of the G maps and the gradient.
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

__device__ __forceinline__ double block_sum(double v, double *sh) {
  for (int d = 32; d > 0; d >>= 1) v += __shfl_xor(v, d, 64);
  const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
  if (lane == 0) sh[wid] = v;
  __syncthreads();
  double t = 0.0;
  if (threadIdx.x == 0)
    for (int w = 0; w < kThreads / 64; ++w) t += sh[w];
  return t;
}

__global__ __launch_bounds__(kThreads) void ssim_stats_kernel(const float *__restrict__ img,
                                                              const float *__restrict__ gt, int W, int H,
                                                              Window win, float c1, float c2,
                                                              float *__restrict__ g1, float *__restrict__ g2,
                                                              float *__restrict__ g3,
                                                              double *__restrict__ partial) {
  __shared__ float sx[kH][kH + 1], sy[kH][kH + 1];
  __shared__ float hz[5][kH][kT + 1];
  __shared__ double sh[kThreads / 64];
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
  double acc = 0.0;
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
    acc += double(S);
    const uint64_t q = off + uint64_t(gy) * W + gx;
    if (g1) {
      g1[q] = 2.f * my * (B - A) / CD - S * (2.f * mx / C - 2.f * mx / D);
      g2[q] = -S / D;
      g3[q] = 2.f * A / CD;
    }
  }
  const double t = block_sum(acc, sh);
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

__global__ __launch_bounds__(kThreads) void ssim_finish_kernel(const double *__restrict__ partial, int nb,
                                                               double n, double scale, float *__restrict__ loss) {
  __shared__ double sh[kThreads / 64];
  double acc = 0.0;
  for (int i = threadIdx.x; i < nb; i += kThreads) acc += partial[i];
  const double t = block_sum(acc, sh);
  if (threadIdx.x == 0) loss[0] = float(scale * (1.0 - t / n));
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
  c.take<double>(nb, &o_part);
  c.take<float>(grad ? 3 * n : 0, &o_g);
  ws->needed = c.used;
  if (!ws->ptr || ws->bytes < ws->needed) return fail(FGS_E_CAPACITY, "workspace too small");
  ws->kind = 0;
  char *b = static_cast<char *>(ws->ptr);
  double *partial = reinterpret_cast<double *>(b + o_part);
  float *g1 = grad ? reinterpret_cast<float *>(b + o_g) : nullptr;
  float *g2 = grad ? g1 + n : nullptr;
  float *g3 = grad ? g2 + n : nullptr;
  Window win;
  double wsum = 0.0, wd[kWin];
  for (int k = 0; k < kWin; ++k) {
    const double d = double(k - kR);
    wd[k] = std::exp(-d * d / (2.0 * 1.5 * 1.5));
    wsum += wd[k];
  }
  for (int k = 0; k < kWin; ++k) win.w[k] = float(wd[k] / wsum);
  hipStream_t s = static_cast<hipStream_t>(stream);
  ssim_stats_kernel<<<grid, kThreads, 0, s>>>(img, gt, W, H, win, c1, c2, g1, g2, g3, partial);
  FGS_LAUNCH_CHECK("ssim_stats_kernel");
  ssim_finish_kernel<<<1, kThreads, 0, s>>>(partial, int(nb), double(n), double(scale), loss);
  FGS_LAUNCH_CHECK("ssim_finish_kernel");
  if (grad) {
    ssim_grad_kernel<<<grid, kThreads, 0, s>>>(img, gt, W, H, win, g1, g2, g3, float(-double(scale) / double(n)),
                                               accumulate, grad);
    FGS_LAUNCH_CHECK("ssim_grad_kernel");
  }
  return FGS_OK;
}
