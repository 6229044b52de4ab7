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
// Two kernels over 16x16 output tiles with a 5-pixel halo staged in LDS,
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
constexpr int kT = 16;             // output tile side (16: 1,024 workgroups per 512^2 view)
constexpr int kH = kT + 2 * kR;    // staged side (26)
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
                                                              float *__restrict__ partial,
                                                              float *__restrict__ partial_l1) {
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
  CompSum acc, acc1;
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
    if (partial_l1) acc1.add(fabsf(sx[r + kR][c + kR] - sy[r + kR][c + kR]));
    const uint64_t q = off + uint64_t(gy) * W + gx;
    if (g1) {
      g1[q] = 2.f * my * (B - A) / CD - S * (2.f * mx / C - 2.f * mx / D);
      g2[q] = -S / D;
      g3[q] = 2.f * A / CD;
    }
  }
  const uint64_t blk = (uint64_t(blockIdx.z) * gridDim.y + blockIdx.y) * gridDim.x + blockIdx.x;
  const float t = block_sum_f32<kThreads>(acc.value(), sh);
  if (threadIdx.x == 0) partial[blk] = t;
  if (partial_l1) {
    __shared__ float sh1[kThreads / 64];  // its own: thread 0 may still read sh
    const float t1 = block_sum_f32<kThreads>(acc1.value(), sh1);
    if (threadIdx.x == 0) partial_l1[blk] = t1;
  }
}

__global__ __launch_bounds__(kThreads) void ssim_grad_kernel(const float *__restrict__ img,
                                                             const float *__restrict__ gt, int W, int H,
                                                             Window win, const float *__restrict__ g1,
                                                             const float *__restrict__ g2,
                                                             const float *__restrict__ g3, float coef,
                                                             int accumulate, float l1_inv_p,
                                                             float *__restrict__ grad) {
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
    const float xq = img[q], yq = gt[q];
    // what the gradient is added to: the image already there, the L1
    // term's sign(x - y) / n_per_view (l1_inv_p > 0; the value the L1
    // kernel writes), or nothing; one rounding in every case
    float base = accumulate ? grad[q] : 0.f;
    if (l1_inv_p > 0.f) {
      const float d = xq - yq;
      base = (d > 0.f) ? l1_inv_p : ((d < 0.f) ? -l1_inv_p : 0.f);
    }
    grad[q] = fmaf(coef, a[0] + 2.f * xq * a[1] + yq * a[2], base);
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

uint64_t ssim_tiles(int32_t W, int32_t H) {
  return uint64_t((W + kT - 1) / kT) * uint64_t((H + kT - 1) / kT);
}

int ssim_l1_partials(const float *img, const float *gt, int32_t W, int32_t H, float c1, float c2, float scale,
                     float l1_inv_p, float *grad, float *gmaps, float *part_ssim, float *part_l1, hipStream_t s) {
  const uint64_t n = uint64_t(W) * uint64_t(H);
  const dim3 grid(unsigned((W + kT - 1) / kT), unsigned((H + kT - 1) / kT), 1u);
  const Window win = gaussian_window();
  ssim_stats_kernel<<<grid, kThreads, 0, s>>>(img, gt, W, H, win, c1, c2, gmaps, gmaps + n, gmaps + 2 * n,
                                              part_ssim, part_l1);
  FGS_LAUNCH_CHECK("ssim_stats_kernel");
  ssim_grad_kernel<<<grid, kThreads, 0, s>>>(img, gt, W, H, win, gmaps, gmaps + n, gmaps + 2 * n,
                                             float(-double(scale) / double(n)), 0, l1_inv_p, grad);
  FGS_LAUNCH_CHECK("ssim_grad_kernel");
  return FGS_OK;
}

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
  ssim_stats_kernel<<<grid, kThreads, 0, s>>>(img, gt, W, H, win, c1, c2, g1, g2, g3, partial, nullptr);
  FGS_LAUNCH_CHECK("ssim_stats_kernel");
  ssim_finish_kernel<<<1, kThreads, 0, s>>>(partial, int(nb), float(double(scale) / double(n)), loss);
  FGS_LAUNCH_CHECK("ssim_finish_kernel");
  if (grad) {
    ssim_grad_kernel<<<grid, kThreads, 0, s>>>(img, gt, W, H, win, g1, g2, g3, float(-double(scale) / double(n)),
                                               accumulate, 0.f, grad);
    FGS_LAUNCH_CHECK("ssim_grad_kernel");
  }
  return FGS_OK;
}

// ---------------------------------------------------------------------------
// 3D SSIM (the fitting loss of Eq. 6): the same per-voxel formula with the
// separable 11^3 window, fused along z with a ring of filtered slices (the
// paper's z-buffered 3D SSIM, Sec. 3.5, laid out for 64-wide wavefronts).
//
// A workgroup owns a 16 x 16 column of voxels over a chunk of kZC output
// slices. It walks the input slices of its chunk (plus the 5-slice halo on
// each side) one at a time: the slice's 26 x 26 neighbourhood is staged in
// LDS, filtered along x, then along y (each thread one column of the 16 x 16
// tile), and the thread keeps the last 11 filtered slices in registers (the
// ring; the loop is unrolled by 11 so every ring slot is a fixed register).
// Once 11 slices are in, the z filter of the middle slice is a weighted sum
// over the ring. Two such kernels:
//   stats: the five statistics from x and y, 1 - SSIM (workgroup partial
//          sums, no atomics) and the three G maps;
//   grad:  the windowed sums of the G maps (same structure, three channels)
//          and the gradient.
// Every filter is x, then y, then z, taps in window order, so the result is
// deterministic.

namespace fgs {
namespace {

constexpr int kST = 16;              // tile side (x, y)
constexpr int kSH = kST + 2 * kR;    // staged side (26)
constexpr int kZC = 64;              // output slices per workgroup
constexpr int kST2 = kST * kST;      // 256 threads, one column each

// The staged neighbourhood of one input slice, held in registers between its
// global loads and its LDS stores: each thread loads kLoads of the slice's
// 26 x 26 positions (IN input arrays each), so that the loads of the next
// slice are in flight while the current one is filtered.
constexpr int kLoads = (kSH * kSH + kST2 - 1) / kST2;  // 3

template <int IN>
struct SliceRegs {
  float v[kLoads][IN];
};

// Global loads of input slice zi (zero outside the grid). IN = 2: arrays a
// and b; else the IN channels a[0..IN) with stride n.
template <int IN>
__device__ __forceinline__ void slice_load(const float *__restrict__ a, const float *__restrict__ b, uint64_t n,
                                           int nx, int ny, int nz, int x0, int y0, int zi, SliceRegs<IN> &r) {
  const bool zin = zi >= 0 && zi < nz;
  const uint64_t zoff = uint64_t(zin ? zi : 0) * uint64_t(nx) * uint64_t(ny);
#pragma unroll
  for (int l = 0; l < kLoads; ++l) {
    const int i = int(threadIdx.x) + l * kST2;
    const int rr = i / kSH, c = i - rr * kSH;
    const int gx = x0 - kR + c, gy = y0 - kR + rr;
    const bool in = zin && i < kSH * kSH && gx >= 0 && gx < nx && gy >= 0 && gy < ny;
    const uint64_t q = zoff + uint64_t(in ? gy : 0) * uint64_t(nx) + uint64_t(in ? gx : 0);
#pragma unroll
    for (int ch = 0; ch < IN; ++ch) {
      const float *src = (IN == 2 && ch == 1) ? b : a + (IN == 2 ? 0 : uint64_t(ch) * n);
      r.v[l][ch] = in ? src[q] : 0.f;
    }
  }
}

// One staged slice through the x and y filters: the thread's column gets
// f[c] for the CH channels. PRODUCTS: channels x, y, x^2, y^2, x y formed
// from the two loaded arrays; else the CH loaded channels. Contains
// barriers: every thread calls it.
template <int CH, bool PRODUCTS, int IN>
__device__ __forceinline__ void slice_filter_2d(const SliceRegs<IN> &r, const Window &win,
                                                float (*sp)[kSH][kSH + 1], float (*sh)[kSH][kST + 1], float f[CH]) {
  __syncthreads();  // the previous slice's reads of sp and sh are done
#pragma unroll
  for (int l = 0; l < kLoads; ++l) {
    const int i = int(threadIdx.x) + l * kST2;
    if (i < kSH * kSH) {
      const int rr = i / kSH, c = i - rr * kSH;
      if (PRODUCTS) {
        const float xv = r.v[l][0], yv = r.v[l][IN - 1];
        sp[0][rr][c] = xv;
        sp[1][rr][c] = yv;
        sp[2][rr][c] = xv * xv;
        sp[3][rr][c] = yv * yv;
        sp[4][rr][c] = xv * yv;
      } else {
#pragma unroll
        for (int ch = 0; ch < CH; ++ch) sp[ch][rr][c] = r.v[l][ch < IN ? ch : 0];
      }
    }
  }
  __syncthreads();
  // x filter: thread t < 208 takes row t / 8 and the two neighbouring
  // outputs c0, c0 + 1 (c0 = 2 (t % 8)), which share 10 of their 11 inputs:
  // 12 LDS reads per channel for two outputs
  if (threadIdx.x < kSH * kST / 2) {
    const int rr = int(threadIdx.x) / (kST / 2), c0 = 2 * (int(threadIdx.x) % (kST / 2));
    // one channel at a time (the ring already holds 11 CH registers)
#pragma unroll 1
    for (int ch = 0; ch < CH; ++ch) {
      float v[kWin + 1];
#pragma unroll
      for (int j = 0; j <= kWin; ++j) v[j] = sp[ch][rr][c0 + j];
      float a0 = 0.f, a1 = 0.f;
#pragma unroll
      for (int k = 0; k < kWin; ++k) {
        a0 = fmaf(win.w[k], v[k], a0);
        a1 = fmaf(win.w[k], v[k + 1], a1);
      }
      sh[ch][rr][c0] = a0;
      sh[ch][rr][c0 + 1] = a1;
    }
  }
  __syncthreads();
  const int tx = threadIdx.x & (kST - 1), ty = threadIdx.x / kST;
#pragma unroll
  for (int ch = 0; ch < CH; ++ch) f[ch] = 0.f;
#pragma unroll
  for (int k = 0; k < kWin; ++k)
#pragma unroll
    for (int ch = 0; ch < CH; ++ch) f[ch] = fmaf(win.w[k], sh[ch][ty + k][tx], f[ch]);
}

// Walks input slices z0 - 5 .. z1 + 4 of the workgroup's chunk [z0, z1): ring
// slot j of the unrolled loop holds input slice base + j. The loads of slice
// k + 1 are issued before slice k is filtered. After the slice k (counted
// from the chunk's first input slice) is filtered, output slice z0 + k - 10
// is complete: emit(zo, m) receives its z-filtered channels.
template <int CH, bool PRODUCTS, int IN, typename Emit>
__device__ __forceinline__ void zring_walk(const float *__restrict__ a, const float *__restrict__ b, uint64_t n,
                                           int nx, int ny, int nz, int x0, int y0, int z0, int z1,
                                           const Window &win, float (*sp)[kSH][kSH + 1],
                                           float (*sh)[kSH][kST + 1], Emit &&emit) {
  float ring[kWin][CH];
  const int n_in = (z1 - z0) + 2 * kR;
  SliceRegs<IN> cur, nxt;
  slice_load<IN>(a, b, n, nx, ny, nz, x0, y0, z0 - kR, cur);
  for (int base = 0; base < n_in; base += kWin) {
#pragma unroll
    for (int j = 0; j < kWin; ++j) {
      const int k = base + j;
      if (k >= n_in) break;  // uniform over the workgroup
      if (k + 1 < n_in) slice_load<IN>(a, b, n, nx, ny, nz, x0, y0, z0 - kR + k + 1, nxt);
      slice_filter_2d<CH, PRODUCTS, IN>(cur, win, sp, sh, ring[j]);
      cur = nxt;
      if (k >= 2 * kR) {
        float m[CH];
#pragma unroll
        for (int ch = 0; ch < CH; ++ch) m[ch] = 0.f;
#pragma unroll
        for (int t = 0; t < kWin; ++t) {
          const int slot = (j + 1 + t) % kWin;  // input slice k - 10 + t
#pragma unroll
          for (int ch = 0; ch < CH; ++ch) m[ch] = fmaf(win.w[t], ring[slot][ch], m[ch]);
        }
        emit(z0 + k - 2 * kR, m);
      }
    }
  }
}

__global__ __launch_bounds__(kST2) void ssim3d_stats_kernel(const float *__restrict__ vol,
                                                            const float *__restrict__ gt, int nx, int ny, int nz,
                                                            Window win, float c1, float c2,
                                                            float *__restrict__ g, float *__restrict__ partial) {
  __shared__ float sp[5][kSH][kSH + 1];
  __shared__ float sh[5][kSH][kST + 1];
  __shared__ float sw[kST2 / 64];
  const uint64_t n = uint64_t(nx) * uint64_t(ny) * uint64_t(nz);
  const int x0 = blockIdx.x * kST, y0 = blockIdx.y * kST;
  const int z0 = blockIdx.z * kZC, z1 = min(z0 + kZC, nz);
  const int X = x0 + int(threadIdx.x & (kST - 1)), Y = y0 + int(threadIdx.x / kST);
  const bool mine = X < nx && Y < ny;
  CompSum acc;
  zring_walk<5, true, 2>(vol, gt, n, nx, ny, nz, x0, y0, z0, z1, win, sp, sh, [&](int zo, const float *m) {
    if (!mine) return;
    const float mx = m[0], my = m[1];
    const float A = fmaf(2.f * mx, my, c1);
    const float B = fmaf(2.f, m[4] - mx * my, c2);
    const float C = fmaf(mx, mx, fmaf(my, my, c1));
    const float D = (m[2] - mx * mx) + (m[3] - my * my) + c2;
    const float CD = C * D;
    const float S = A * B / CD;
    acc.add(1.f - S);
    if (g) {
      const uint64_t q = (uint64_t(zo) * uint64_t(ny) + uint64_t(Y)) * uint64_t(nx) + uint64_t(X);
      g[q] = 2.f * my * (B - A) / CD - S * (2.f * mx / C - 2.f * mx / D);
      g[n + q] = -S / D;
      g[2 * n + q] = 2.f * A / CD;
    }
  });
  const float t = block_sum_f32<kST2>(acc.value(), sw);
  if (threadIdx.x == 0) partial[(uint64_t(blockIdx.z) * gridDim.y + blockIdx.y) * gridDim.x + blockIdx.x] = t;
}

__global__ __launch_bounds__(kST2) void ssim3d_grad_kernel(const float *__restrict__ vol,
                                                           const float *__restrict__ gt, int nx, int ny, int nz,
                                                           Window win, const float *__restrict__ g, float coef,
                                                           int accumulate, float *__restrict__ grad) {
  __shared__ float sp[3][kSH][kSH + 1];
  __shared__ float sh[3][kSH][kST + 1];
  const uint64_t n = uint64_t(nx) * uint64_t(ny) * uint64_t(nz);
  const int x0 = blockIdx.x * kST, y0 = blockIdx.y * kST;
  const int z0 = blockIdx.z * kZC, z1 = min(z0 + kZC, nz);
  const int X = x0 + int(threadIdx.x & (kST - 1)), Y = y0 + int(threadIdx.x / kST);
  const bool mine = X < nx && Y < ny;
  zring_walk<3, false, 3>(g, nullptr, n, nx, ny, nz, x0, y0, z0, z1, win, sp, sh, [&](int zo, const float *m) {
    if (!mine) return;
    const uint64_t q = (uint64_t(zo) * uint64_t(ny) + uint64_t(Y)) * uint64_t(nx) + uint64_t(X);
    const float gq = coef * (m[0] + 2.f * vol[q] * m[1] + gt[q] * m[2]);
    grad[q] = accumulate ? grad[q] + gq : gq;
  });
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
  const dim3 grid(unsigned((nx + kST - 1) / kST), unsigned((ny + kST - 1) / kST), unsigned((nz + kZC - 1) / kZC));
  if (grid.y > 65535 || grid.z > 65535) return fail(FGS_E_UNSUPPORTED, "grid too large");
  const uint64_t nb = uint64_t(grid.x) * grid.y * grid.z;
  Carver c(nullptr);
  uint64_t o_g, o_part;
  c.take<float>(grad ? 3 * n : 0, &o_g);
  c.take<float>(nb, &o_part);
  ws->needed = c.used;
  if (!ws->ptr || ws->bytes < ws->needed) return fail(FGS_E_CAPACITY, "workspace too small");
  ws->kind = 0;
  char *b = static_cast<char *>(ws->ptr);
  float *g = grad ? reinterpret_cast<float *>(b + o_g) : nullptr;
  float *partial = reinterpret_cast<float *>(b + o_part);
  const Window win = gaussian_window();
  hipStream_t s = static_cast<hipStream_t>(stream);
  ssim3d_stats_kernel<<<grid, kST2, 0, s>>>(vol, gt, nx, ny, nz, win, c1, c2, g, partial);
  FGS_LAUNCH_CHECK("ssim3d_stats_kernel");
  ssim_finish_kernel<<<1, kThreads, 0, s>>>(partial, int(nb), float(double(scale) / double(n)), loss);
  FGS_LAUNCH_CHECK("ssim_finish_kernel");
  if (grad) {
    ssim3d_grad_kernel<<<grid, kST2, 0, s>>>(vol, gt, nx, ny, nz, win, g, float(-double(scale) / double(n)),
                                             accumulate, grad);
    FGS_LAUNCH_CHECK("ssim3d_grad_kernel");
  }
  return FGS_OK;
}
