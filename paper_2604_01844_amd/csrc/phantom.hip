// Additive ellipsoid phantom in FP64: exact chord projections along the same
// cone-beam / parallel-beam rays the rasterizer samples, and the indicator
// sum at voxel centres. Synthetic ground truth that stands in for the
// paper's datasets (Sec. 4.1 uses real volumes with simulated projections).
// Each ellipsoid is handled in its own frame: x' = diag(1/a) R^T (x - c),
// inside iff |x'|^2 <= 1; along a ray o + t d the chord length is
// 2 sqrt(B^2 - A C) / A with A = |d'|^2, B = o'.d', C = |o'|^2 - 1.
#include "fgs_internal.h"

namespace fgs {
namespace {

constexpr int kChunk = 128;

struct EllDev {
  double M[9];   // diag(1/a) R^T, row-major
  double c[3];
  double amp;
};

__device__ void load_ellipsoid(const fgs_phantom &ph, int64_t e, EllDev &E) {
  const double *q = ph.quat + 4 * e;
  const double n = sqrt(q[0] * q[0] + q[1] * q[1] + q[2] * q[2] + q[3] * q[3]);
  const double w = q[0] / n, x = q[1] / n, y = q[2] / n, z = q[3] / n;
  const double R[9] = {1 - 2 * (y * y + z * z), 2 * (x * y - w * z),     2 * (x * z + w * y),
                       2 * (x * y + w * z),     1 - 2 * (x * x + z * z), 2 * (y * z - w * x),
                       2 * (x * z - w * y),     2 * (y * z + w * x),     1 - 2 * (x * x + y * y)};
  for (int j = 0; j < 3; ++j) {
    const double ia = 1.0 / ph.semi[3 * e + j];
    for (int a = 0; a < 3; ++a) E.M[3 * j + a] = R[3 * a + j] * ia;  // row j = column j of R / a_j
    E.c[j] = ph.centre[3 * e + j];
  }
  E.amp = ph.amp[e];
}

__global__ __launch_bounds__(256) void phantom_project_kernel(fgs_phantom ph, fgs_geom g, int view_begin,
                                                              float *__restrict__ img) {
  __shared__ EllDev s_e[kChunk];
  const int v_local = blockIdx.y;
  const int64_t pix = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  const int64_t np = int64_t(g.det_w) * g.det_h;
  const double th = double(g.angles[view_begin + v_local]);
  const double sn = sin(th), cs = cos(th);
  const double e0[3] = {-sn, cs, 0.0}, e1[3] = {0.0, 0.0, -1.0}, e2[3] = {-cs, -sn, 0.0};
  const int px = int(pix % g.det_w), py = int(pix / g.det_w);
  const double xu = (px + 0.5 - (0.5 * g.det_w + double(g.off_u))) * double(g.pitch_u);
  const double xv = (py + 0.5 - (0.5 * g.det_h + double(g.off_v))) * double(g.pitch_v);
  double o[3], d[3];
  if (g.mode == FGS_CONE) {
    double nn = 0.0;
    for (int a = 0; a < 3; ++a) {
      o[a] = (a == 0 ? cs : (a == 1 ? sn : 0.0)) * double(g.sod);
      d[a] = double(g.sdd) * e2[a] + xu * e0[a] + xv * e1[a];
      nn += d[a] * d[a];
    }
    nn = 1.0 / sqrt(nn);
    for (int a = 0; a < 3; ++a) d[a] *= nn;
  } else {
    for (int a = 0; a < 3; ++a) {
      o[a] = xu * e0[a] + xv * e1[a] - 2.0 * e2[a];
      d[a] = e2[a];
    }
  }
  double acc = 0.0;
  for (int64_t base = 0; base < ph.n; base += kChunk) {
    const int m = int(min(int64_t(kChunk), ph.n - base));
    __syncthreads();
    for (int k = threadIdx.x; k < m; k += blockDim.x) load_ellipsoid(ph, base + k, s_e[k]);
    __syncthreads();
    for (int k = 0; k < m; ++k) {
      const EllDev &E = s_e[k];
      double op[3], dp[3];
      for (int j = 0; j < 3; ++j) {
        op[j] = E.M[3 * j] * (o[0] - E.c[0]) + E.M[3 * j + 1] * (o[1] - E.c[1]) + E.M[3 * j + 2] * (o[2] - E.c[2]);
        dp[j] = E.M[3 * j] * d[0] + E.M[3 * j + 1] * d[1] + E.M[3 * j + 2] * d[2];
      }
      const double A = dp[0] * dp[0] + dp[1] * dp[1] + dp[2] * dp[2];
      const double B = op[0] * dp[0] + op[1] * dp[1] + op[2] * dp[2];
      const double C = op[0] * op[0] + op[1] * op[1] + op[2] * op[2] - 1.0;
      const double disc = B * B - A * C;
      if (disc > 0.0) acc += E.amp * 2.0 * sqrt(disc) / A;
    }
  }
  if (pix < np) img[int64_t(v_local) * np + pix] = float(acc);
}

__global__ __launch_bounds__(256) void phantom_volume_kernel(fgs_phantom ph, fgs_grid gr,
                                                             float *__restrict__ vol) {
  __shared__ EllDev s_e[kChunk];
  const int64_t idx = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  const int64_t nx = gr.dims[0], ny = gr.dims[1], nz = gr.dims[2];
  const int64_t ix = idx % nx, iy = (idx / nx) % ny, iz = idx / (nx * ny);
  const double x[3] = {double(gr.origin[0]) + (ix + 0.5) * double(gr.spacing[0]),
                       double(gr.origin[1]) + (iy + 0.5) * double(gr.spacing[1]),
                       double(gr.origin[2]) + (iz + 0.5) * double(gr.spacing[2])};
  double acc = 0.0;
  for (int64_t base = 0; base < ph.n; base += kChunk) {
    const int m = int(min(int64_t(kChunk), ph.n - base));
    __syncthreads();
    for (int k = threadIdx.x; k < m; k += blockDim.x) load_ellipsoid(ph, base + k, s_e[k]);
    __syncthreads();
    for (int k = 0; k < m; ++k) {
      const EllDev &E = s_e[k];
      double r2 = 0.0;
      for (int j = 0; j < 3; ++j) {
        const double y = E.M[3 * j] * (x[0] - E.c[0]) + E.M[3 * j + 1] * (x[1] - E.c[1]) +
                         E.M[3 * j + 2] * (x[2] - E.c[2]);
        r2 += y * y;
      }
      if (r2 <= 1.0) acc += E.amp;
    }
  }
  if (idx < nx * ny * nz) vol[idx] = float(acc);
}

}  // namespace
}  // namespace fgs

using namespace fgs;

extern "C" int fgs_phantom_project(const fgs_phantom *ph, const fgs_geom *geom, int32_t view_begin,
                                   int32_t view_count, float *img, void *stream) {
  if (!ph || !geom || !img || !ph->centre || !ph->semi || !ph->quat || !ph->amp || !geom->angles)
    return fail(FGS_E_INVALID, "null argument");
  if (ph->n <= 0 || geom->det_w <= 0 || geom->det_h <= 0 || view_count <= 0 || view_begin < 0 ||
      int64_t(view_begin) + view_count > geom->n_views)
    return fail(FGS_E_INVALID, "sizes or view range");
  hipStream_t s = static_cast<hipStream_t>(stream);
  const uint64_t np = uint64_t(geom->det_w) * geom->det_h;
  dim3 grid(grid_for(np, 256), unsigned(view_count));
  phantom_project_kernel<<<grid, 256, 0, s>>>(*ph, *geom, view_begin, img);
  FGS_LAUNCH_CHECK("phantom_project_kernel");
  return FGS_OK;
}

extern "C" int fgs_phantom_voxelize(const fgs_phantom *ph, const fgs_grid *grid, float *vol, void *stream) {
  if (!ph || !grid || !vol || !ph->centre || !ph->semi || !ph->quat || !ph->amp)
    return fail(FGS_E_INVALID, "null argument");
  if (ph->n <= 0 || grid->dims[0] <= 0 || grid->dims[1] <= 0 || grid->dims[2] <= 0)
    return fail(FGS_E_INVALID, "sizes");
  hipStream_t s = static_cast<hipStream_t>(stream);
  const uint64_t nv = uint64_t(grid->dims[0]) * grid->dims[1] * grid->dims[2];
  phantom_volume_kernel<<<grid_for(nv, 256), 256, 0, s>>>(*ph, *grid, vol);
  FGS_LAUNCH_CHECK("phantom_volume_kernel");
  return FGS_OK;
}
