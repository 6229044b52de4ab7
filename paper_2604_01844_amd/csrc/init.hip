// Initialisation path of the reconstruction (Sec. 3.1): an FDK
// reconstruction of the projections, then Gaussian means sampled with
// probability proportional to the gradient magnitude of the
// background-thresholded FDK volume, densities k times the FDK intensity at
// the sample, zero rotation, scale equal to the nearest-neighbour distance.
//
// FDK (Feldkamp, Davis and Kress) for a full circular scan on a flat
// detector, discretised on the detector rescaled to the rotation axis
// (pitch p' = pitch * sod / sdd, coordinates a', b'):
//   weight    pw = p * sod / sqrt(sod^2 + a'^2 + b'^2)
//   filter    q[n] = p' sum_k h[n - k] pw[k],  h[0] = 1 / (4 p'^2),
//             h[m odd] = -1 / (pi^2 m^2 p'^2), h[m even] = 0  (Ram-Lak)
//   backproject f(x) = 1/2 * (2 pi / V) * sum_views (sod / t2)^2 q(u(x), v(x))
// with t2 the depth of x along the central ray, (u, v) the detector pixel
// coordinates of x's projection (the rasterizer's camera model), bilinear
// interpolation between pixel centres and zero outside the detector.
//
// Sampling is exact in integers: per-voxel weights are the FP32 gradient
// magnitude (or, for intensity sampling, the thresholded value) quantised to
// 24 bits of its maximum, their 64-bit prefix sum is
// the CDF, and draw i takes the voxel whose CDF interval holds
// floor(u_i * total) (u_i given, FP64).
#include <cmath>

#include "fgs_internal.h"

namespace fgs {
namespace {

constexpr int kMaxFilterRow = 8192;

__global__ __launch_bounds__(256) void fdk_filter_kernel(const float *__restrict__ img, int W, int H,
                                                         float sod, float pu, float pv, float cu, float cv,
                                                         float *__restrict__ q) {
  __shared__ float row[kMaxFilterRow];
  const int v_local = blockIdx.y;
  const int i = blockIdx.x;
  const float *src = img + (uint64_t(v_local) * H + i) * uint64_t(W);
  const float b = (float(i) + 0.5f - cv) * pv;
  for (int j = threadIdx.x; j < W; j += blockDim.x) {
    const float a = (float(j) + 0.5f - cu) * pu;
    row[j] = src[j] * sod / sqrtf(sod * sod + a * a + b * b);
  }
  __syncthreads();
  const float pi2 = 9.8696044010893586f;
  const float inv = 1.f / (pu * pu);
  float *dst = q + (uint64_t(v_local) * H + i) * uint64_t(W);
  for (int n = threadIdx.x; n < W; n += blockDim.x) {
    float acc = 0.25f * inv * row[n];
    for (int m = 1; m < W; m += 2) {
      const float hm = -inv / (pi2 * float(m) * float(m));
      const float l = (n - m >= 0) ? row[n - m] : 0.f;
      const float r = (n + m < W) ? row[n + m] : 0.f;
      acc = fmaf(hm, l + r, acc);
    }
    dst[n] = pu * acc;
  }
}

struct FdkGeom {
  float sod, fu, fv, cu, cv;
  int W, H, views, view_begin;
  float scale;  // 1/2 * 2 pi / V
  const float *angles;
  float origin[3], h[3];
  int dims[3];
};

__global__ __launch_bounds__(256) void fdk_backproject_kernel(FdkGeom G, const float *__restrict__ q,
                                                              float *__restrict__ vol) {
  __shared__ float s_cs[1024][2];
  for (int v = threadIdx.x; v < G.views; v += blockDim.x) {
    float sn, cs;
    sincosf(G.angles[G.view_begin + v], &sn, &cs);
    s_cs[v][0] = cs;
    s_cs[v][1] = sn;
  }
  __syncthreads();
  const int64_t nvox = int64_t(G.dims[0]) * G.dims[1] * G.dims[2];
  const int64_t idx = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (idx >= nvox) return;
  const int ix = int(idx % G.dims[0]);
  const int iy = int((idx / G.dims[0]) % G.dims[1]);
  const int iz = int(idx / (int64_t(G.dims[0]) * G.dims[1]));
  const float x = G.origin[0] + (float(ix) + 0.5f) * G.h[0];
  const float y = G.origin[1] + (float(iy) + 0.5f) * G.h[1];
  const float z = G.origin[2] + (float(iz) + 0.5f) * G.h[2];
  float acc = 0.f;
  for (int v = 0; v < G.views; ++v) {
    const float c = s_cs[v][0], s = s_cs[v][1];
    // t = W (x - src), rows e0 = (-s, c, 0), e1 = (0, 0, -1), e2 = (-c, -s, 0)
    const float dx = x - G.sod * c, dy = y - G.sod * s;
    const float t0 = -s * dx + c * dy;
    const float t1 = -z;
    const float t2 = -c * dx - s * dy;
    if (!(t2 > 0.f)) continue;
    const float it = 1.f / t2;
    const float u = G.fu * t0 * it + G.cu - 0.5f;
    const float w = G.fv * t1 * it + G.cv - 0.5f;
    const float u0f = floorf(u), w0f = floorf(w);
    const int u0 = int(u0f), w0 = int(w0f);
    const float fu = u - u0f, fw = w - w0f;
    const float *qv = q + uint64_t(v) * G.H * uint64_t(G.W);
    auto at = [&](int uu, int ww) -> float {
      return (uu >= 0 && uu < G.W && ww >= 0 && ww < G.H) ? qv[uint64_t(ww) * G.W + uu] : 0.f;
    };
    const float val = (1.f - fw) * ((1.f - fu) * at(u0, w0) + fu * at(u0 + 1, w0)) +
                      fw * ((1.f - fu) * at(u0, w0 + 1) + fu * at(u0 + 1, w0 + 1));
    const float wt = G.sod * it;
    acc = fmaf(wt * wt, val, acc);
  }
  vol[idx] = G.scale * acc;
}

// ------------------------------------------------------------ init sampling

constexpr int kRedThreads = 256;
constexpr int kRedBlocks = 1024;

__global__ __launch_bounds__(kRedThreads) void max_partial_kernel(const float *__restrict__ a, uint64_t n,
                                                                  float *__restrict__ partial) {
  __shared__ float sh[kRedThreads / 64];
  float m = -INFINITY;
  for (uint64_t i = uint64_t(blockIdx.x) * kRedThreads + threadIdx.x; i < n; i += uint64_t(gridDim.x) * kRedThreads)
    m = fmaxf(m, a[i]);
  for (int d = 32; d > 0; d >>= 1) m = fmaxf(m, __shfl_xor(m, d, 64));
  if ((threadIdx.x & 63) == 0) sh[threadIdx.x >> 6] = m;
  __syncthreads();
  if (threadIdx.x == 0) {
    float t = sh[0];
    for (int w = 1; w < kRedThreads / 64; ++w) t = fmaxf(t, sh[w]);
    partial[blockIdx.x] = t;
  }
}

__global__ __launch_bounds__(kRedThreads) void max_final_kernel(const float *__restrict__ partial, int nb,
                                                                float *__restrict__ dst) {
  __shared__ float sh[kRedThreads / 64];
  float m = -INFINITY;
  for (int i = threadIdx.x; i < nb; i += kRedThreads) m = fmaxf(m, partial[i]);
  for (int d = 32; d > 0; d >>= 1) m = fmaxf(m, __shfl_xor(m, d, 64));
  if ((threadIdx.x & 63) == 0) sh[threadIdx.x >> 6] = m;
  __syncthreads();
  if (threadIdx.x == 0) {
    float t = sh[0];
    for (int w = 1; w < kRedThreads / 64; ++w) t = fmaxf(t, sh[w]);
    dst[0] = t;
  }
}

// Gradient magnitude (central differences, zero outside the grid) of the
// volume with voxels below background_fraction * max set to zero.
__global__ __launch_bounds__(256) void grad_mag_kernel(const float *__restrict__ vol, int nx, int ny, int nz,
                                                       float background_fraction,
                                                       const float *__restrict__ vmax,
                                                       float *__restrict__ gmag) {
#pragma clang fp contract(off)
  const int64_t idx = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  const int64_t nv = int64_t(nx) * ny * nz;
  if (idx >= nv) return;
  const float thr = background_fraction * vmax[0];
  const int ix = int(idx % nx), iy = int((idx / nx) % ny), iz = int(idx / (int64_t(nx) * ny));
  auto val = [&](int x, int y, int z) -> float {
    if (x < 0 || x >= nx || y < 0 || y >= ny || z < 0 || z >= nz) return 0.f;
    const float v = vol[(int64_t(z) * ny + y) * nx + x];
    return (v >= thr) ? v : 0.f;
  };
  const float gx = 0.5f * (val(ix + 1, iy, iz) - val(ix - 1, iy, iz));
  const float gy = 0.5f * (val(ix, iy + 1, iz) - val(ix, iy - 1, iz));
  const float gz = 0.5f * (val(ix, iy, iz + 1) - val(ix, iy, iz - 1));
  const float sq = gx * gx + gy * gy;
  gmag[idx] = sqrtf(sq + gz * gz);
}

// Intensity weighting: the volume itself with voxels below
// background_fraction * max (and negative values) set to zero.
__global__ __launch_bounds__(256) void intensity_kernel(const float *__restrict__ vol, uint64_t nv,
                                                        float background_fraction,
                                                        const float *__restrict__ vmax,
                                                        float *__restrict__ wgt) {
  const uint64_t idx = uint64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (idx >= nv) return;
  const float thr = background_fraction * vmax[0];
  const float v = vol[idx];
  wgt[idx] = (v >= thr && v > 0.f) ? v : 0.f;
}

__global__ __launch_bounds__(256) void quantize_kernel(const float *__restrict__ gmag, uint64_t n,
                                                       const float *__restrict__ gmax,
                                                       uint64_t *__restrict__ w) {
#pragma clang fp contract(off)
  const uint64_t i = uint64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const float scale = 16777216.f / gmax[0];
  w[i] = static_cast<uint64_t>(floorf(gmag[i] * scale));
}

__device__ __forceinline__ float trilinear(const float *__restrict__ vol, const int dims[3], const float c[3]) {
  const float f0 = floorf(c[0]), f1 = floorf(c[1]), f2 = floorf(c[2]);
  const int i0 = int(f0), j0 = int(f1), k0 = int(f2);
  const float a = c[0] - f0, b = c[1] - f1, g = c[2] - f2;
  float acc = 0.f;
  for (int dz = 0; dz < 2; ++dz)
    for (int dy = 0; dy < 2; ++dy)
      for (int dx = 0; dx < 2; ++dx) {
        const int x = i0 + dx, y = j0 + dy, z = k0 + dz;
        if (x < 0 || x >= dims[0] || y < 0 || y >= dims[1] || z < 0 || z >= dims[2]) continue;
        const float wgt = (dx ? a : 1.f - a) * (dy ? b : 1.f - b) * (dz ? g : 1.f - g);
        acc = fmaf(wgt, vol[(int64_t(z) * dims[1] + y) * dims[0] + x], acc);
      }
  return acc;
}

struct InitGrid {
  float origin[3], h[3];
  int dims[3];
};

__global__ __launch_bounds__(256) void sample_kernel(const uint64_t *__restrict__ cdf, uint64_t nvox,
                                                     const float *__restrict__ vol, InitGrid G,
                                                     const double *__restrict__ uni, int64_t n,
                                                     float density_scale, fgs_gaussian_grads out) {
  const int64_t i = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const uint64_t total = cdf[nvox];
  uint64_t target = static_cast<uint64_t>(floor(uni[i] * double(total)));
  if (target >= total) target = total - 1;
  // largest k with cdf[k] <= target (cdf is non-decreasing, cdf[0] = 0)
  uint64_t lo = 0, hi = nvox;  // invariant: cdf[lo] <= target < cdf[hi] (cdf[nvox] = total > target)
  while (hi - lo > 1) {
    const uint64_t mid = (lo + hi) >> 1;
    if (cdf[mid] <= target)
      lo = mid;
    else
      hi = mid;
  }
  const int64_t k = int64_t(lo);
  const int ix = int(k % G.dims[0]), iy = int((k / G.dims[0]) % G.dims[1]),
            iz = int(k / (int64_t(G.dims[0]) * G.dims[1]));
  const int idx3[3] = {ix, iy, iz};
  float p[3], c[3];
  for (int a = 0; a < 3; ++a) {
    const double j = uni[(a + 1) * n + i];
    p[a] = float(double(G.origin[a]) + (double(idx3[a]) + j) * double(G.h[a]));
    c[a] = float(double(idx3[a]) + j - 0.5);
  }
  const float rho = density_scale * trilinear(vol, G.dims, c);
  for (int a = 0; a < 3; ++a) out.mean[a * n + i] = p[a];
  out.quat[i] = 1.f;
  out.quat[n + i] = 0.f;
  out.quat[2 * n + i] = 0.f;
  out.quat[3 * n + i] = 0.f;
  out.density[i] = rho;
}

// Isotropic log-scale = log of the distance to the nearest other mean
// (brute force over LDS tiles), floored at min_dist.
__global__ __launch_bounds__(256) void nn_scale_kernel(const float *__restrict__ mean, int64_t n,
                                                       float min_dist, float *__restrict__ log_scale) {
  __shared__ float s_p[3][256];
  const int64_t i = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  float px = 0.f, py = 0.f, pz = 0.f;
  if (i < n) {
    px = mean[i];
    py = mean[n + i];
    pz = mean[2 * n + i];
  }
  float best = INFINITY;
  for (int64_t base = 0; base < n; base += 256) {
    __syncthreads();
    const int64_t j = base + threadIdx.x;
    if (j < n) {
      s_p[0][threadIdx.x] = mean[j];
      s_p[1][threadIdx.x] = mean[n + j];
      s_p[2][threadIdx.x] = mean[2 * n + j];
    }
    __syncthreads();
    const int m = int(min(int64_t(256), n - base));
    for (int t = 0; t < m; ++t) {
      const float dx = s_p[0][t] - px, dy = s_p[1][t] - py, dz = s_p[2][t] - pz;
      const float d2 = fmaf(dx, dx, fmaf(dy, dy, dz * dz));
      best = (base + t != i) ? fminf(best, d2) : best;
    }
  }
  if (i < n) {
    const float d = fmaxf(sqrtf(best), min_dist);
    const float l = logf(d);
    log_scale[i] = l;
    log_scale[n + i] = l;
    log_scale[2 * n + i] = l;
  }
}

}  // namespace
}  // namespace fgs

using namespace fgs;

extern "C" int fgs_fdk(const float *img, const fgs_geom *geom, int32_t view_begin, int32_t view_count,
                       const fgs_grid *grid, float *vol, fgs_workspace *ws, void *stream) {
  if (!img || !geom || !grid || !vol || !ws || !geom->angles) return fail(FGS_E_INVALID, "null argument");
  if (geom->mode != FGS_CONE) return fail(FGS_E_UNSUPPORTED, "FDK is implemented for cone beam only");
  if (view_count <= 0 || view_count > 1024 || view_begin < 0 || int64_t(view_begin) + view_count > geom->n_views)
    return fail(FGS_E_INVALID, "view range (at most 1024 views)");
  if (geom->det_w <= 0 || geom->det_w > kMaxFilterRow || geom->det_h <= 0)
    return fail(FGS_E_INVALID, "detector size (rows up to 8192 pixels)");
  for (int a = 0; a < 3; ++a)
    if (grid->dims[a] <= 0 || !(grid->spacing[a] > 0.f)) return fail(FGS_E_INVALID, "grid");
  const uint64_t qn = uint64_t(view_count) * geom->det_h * geom->det_w;
  ws->needed = align_up(qn * sizeof(float));
  if (!ws->ptr || ws->bytes < ws->needed) return fail(FGS_E_CAPACITY, "workspace too small");
  ws->kind = 0;
  hipStream_t s = static_cast<hipStream_t>(stream);
  float *q = static_cast<float *>(ws->ptr);
  const float ratio = geom->sod / geom->sdd;
  const float cu = 0.5f * float(geom->det_w) + geom->off_u, cv = 0.5f * float(geom->det_h) + geom->off_v;
  dim3 fgrid(unsigned(geom->det_h), unsigned(view_count));
  fdk_filter_kernel<<<fgrid, 256, 0, s>>>(img, geom->det_w, geom->det_h, geom->sod, geom->pitch_u * ratio,
                                          geom->pitch_v * ratio, cu, cv, q);
  FGS_LAUNCH_CHECK("fdk_filter_kernel");
  FdkGeom G{};
  G.sod = geom->sod;
  G.fu = geom->sdd / geom->pitch_u;
  G.fv = geom->sdd / geom->pitch_v;
  G.cu = cu;
  G.cv = cv;
  G.W = geom->det_w;
  G.H = geom->det_h;
  G.views = view_count;
  G.view_begin = view_begin;
  G.scale = float(M_PI / double(view_count));
  G.angles = geom->angles;
  for (int a = 0; a < 3; ++a) {
    G.origin[a] = grid->origin[a];
    G.h[a] = grid->spacing[a];
    G.dims[a] = grid->dims[a];
  }
  const uint64_t nv = uint64_t(grid->dims[0]) * grid->dims[1] * grid->dims[2];
  fdk_backproject_kernel<<<grid_for(nv, 256), 256, 0, s>>>(G, q, vol);
  FGS_LAUNCH_CHECK("fdk_backproject_kernel");
  return FGS_OK;
}

enum class Weighting { kGradient, kIntensity };

static int sampling_init(Weighting mode, const float *vol, const fgs_grid *grid, float background_fraction,
                         float density_scale, float min_scale, int64_t n, const double *uniforms,
                         fgs_gaussians_out *out, fgs_workspace *ws, void *stream) {
  if (!vol || !grid || !uniforms || !out || !ws || !out->mean || !out->log_scale || !out->quat || !out->density)
    return fail(FGS_E_INVALID, "null argument");
  if (n <= 0) return fail(FGS_E_INVALID, "n must be positive");
  for (int a = 0; a < 3; ++a)
    if (grid->dims[a] <= 0 || !(grid->spacing[a] > 0.f)) return fail(FGS_E_INVALID, "grid");
  const uint64_t nv = uint64_t(grid->dims[0]) * grid->dims[1] * grid->dims[2];
  Carver c(nullptr);
  uint64_t o_part, o_g, o_w, o_scan;
  c.take<float>(kRedBlocks + 2, &o_part);
  c.take<float>(nv, &o_g);
  c.take<uint64_t>(nv + 1, &o_w);
  c.take<uint32_t>(scan_scratch_words(nv), &o_scan);
  ws->needed = c.used;
  if (!ws->ptr || ws->bytes < ws->needed) return fail(FGS_E_CAPACITY, "workspace too small");
  ws->kind = 0;
  hipStream_t s = static_cast<hipStream_t>(stream);
  char *b = static_cast<char *>(ws->ptr);
  float *part = reinterpret_cast<float *>(b + o_part);
  float *vmax = part + kRedBlocks;       // holds max(vol)
  float *gmax = part + kRedBlocks + 1;   // holds max(gradient magnitude)
  float *gmag = reinterpret_cast<float *>(b + o_g);
  uint64_t *w = reinterpret_cast<uint64_t *>(b + o_w);
  const int nb = int(std::min<uint64_t>(kRedBlocks, (nv + kRedThreads - 1) / kRedThreads));
  max_partial_kernel<<<nb, kRedThreads, 0, s>>>(vol, nv, part);
  max_final_kernel<<<1, kRedThreads, 0, s>>>(part, nb, vmax);
  FGS_LAUNCH_CHECK("max_final_kernel");
  if (mode == Weighting::kGradient) {
    grad_mag_kernel<<<grid_for(nv, 256), 256, 0, s>>>(vol, grid->dims[0], grid->dims[1], grid->dims[2],
                                                      background_fraction, vmax, gmag);
    FGS_LAUNCH_CHECK("grad_mag_kernel");
  } else {
    intensity_kernel<<<grid_for(nv, 256), 256, 0, s>>>(vol, nv, background_fraction, vmax, gmag);
    FGS_LAUNCH_CHECK("intensity_kernel");
  }
  max_partial_kernel<<<nb, kRedThreads, 0, s>>>(gmag, nv, part);
  max_final_kernel<<<1, kRedThreads, 0, s>>>(part, nb, gmax);
  FGS_LAUNCH_CHECK("max_final_kernel");
  float gm_host = 0.f;
  FGS_HIP(hipMemcpyAsync(&gm_host, gmax, sizeof(float), hipMemcpyDeviceToHost, s));
  FGS_HIP(hipStreamSynchronize(s));
  if (!(gm_host > 0.f))
    return fail(FGS_E_INVALID, mode == Weighting::kGradient ? "the thresholded volume has no gradient to sample"
                                                            : "the thresholded volume has no mass to sample");
  quantize_kernel<<<grid_for(nv, 256), 256, 0, s>>>(gmag, nv, gmax, w);
  FGS_LAUNCH_CHECK("quantize_kernel");
  int st = exclusive_scan_u64(w, nv, reinterpret_cast<uint32_t *>(b + o_scan), s);
  if (st != FGS_OK) return st;
  InitGrid G{};
  for (int a = 0; a < 3; ++a) {
    G.origin[a] = grid->origin[a];
    G.h[a] = grid->spacing[a];
    G.dims[a] = grid->dims[a];
  }
  sample_kernel<<<grid_for(uint64_t(n), 256), 256, 0, s>>>(w, nv, vol, G, uniforms, n, density_scale, *out);
  FGS_LAUNCH_CHECK("sample_kernel");
  nn_scale_kernel<<<grid_for(uint64_t(n), 256), 256, 0, s>>>(out->mean, n, min_scale, out->log_scale);
  FGS_LAUNCH_CHECK("nn_scale_kernel");
  return FGS_OK;
}

extern "C" int fgs_gradient_init(const float *vol, const fgs_grid *grid, float background_fraction,
                                 float density_scale, float min_scale, int64_t n, const double *uniforms,
                                 fgs_gaussians_out *out, fgs_workspace *ws, void *stream) {
  return sampling_init(Weighting::kGradient, vol, grid, background_fraction, density_scale, min_scale, n,
                       uniforms, out, ws, stream);
}

extern "C" int fgs_intensity_init(const float *vol, const fgs_grid *grid, float background_fraction,
                                  float density_scale, float min_scale, int64_t n, const double *uniforms,
                                  fgs_gaussians_out *out, fgs_workspace *ws, void *stream) {
  return sampling_init(Weighting::kIntensity, vol, grid, background_fraction, density_scale, min_scale, n,
                       uniforms, out, ws, stream);
}

extern "C" int fgs_reduce_max(const float *x, int64_t n, float *out, fgs_workspace *ws, void *stream) {
  if (!x || !out || !ws || n <= 0) return fail(FGS_E_INVALID, "invalid argument");
  ws->needed = uint64_t(kRedBlocks) * sizeof(float);
  if (!ws->ptr || ws->bytes < ws->needed) return fail(FGS_E_CAPACITY, "workspace too small");
  ws->kind = 0;
  hipStream_t s = static_cast<hipStream_t>(stream);
  float *part = static_cast<float *>(ws->ptr);
  const int nb = int(std::min<uint64_t>(kRedBlocks, (uint64_t(n) + kRedThreads - 1) / kRedThreads));
  max_partial_kernel<<<nb, kRedThreads, 0, s>>>(x, uint64_t(n), part);
  max_final_kernel<<<1, kRedThreads, 0, s>>>(part, nb, out);
  FGS_LAUNCH_CHECK("max_final_kernel");
  return FGS_OK;
}
