// fgs_recon_step: one optimiser step of the reconstruction loop (Sec. 3.4),
// the paper's unit of work, composed natively so that a step costs one call
// from the host instead of about twenty:
//   rasterizer forward of one view -> L1 (+ SSIM) of Eq. 5 against the
//   measured view, gradient image -> rasterizer backward (lists reused) ->
//   optionally a crop of the grid voxelized, its TV gradient and the
//   voxelizer backward added in -> one Adam launch over all 11 N parameters.
// With key_capacity set in both rasterizer and crop workspaces nothing in the
// step waits for the GPU, so the host runs ahead and a sequence of steps can
// be captured in a HIP graph.
#include <cmath>

#include "fgs_internal.h"

namespace fgs {
namespace {

// Adam (with bias correction) on the four parameter groups in one launch:
// blockIdx.y is the parameter row (3 mean, 3 log-scale, 4 quaternion, 1
// density rows of n values); density is clamped at zero. The arithmetic is
// that of fgs_adam_step, so the result is the same bit for bit.
struct AdamGroups {
  float *p[4];
  const float *g[4];
  float *m[4], *v[4];
  float lr[4];
};

__global__ __launch_bounds__(256) void adam_groups_kernel(AdamGroups A, uint64_t n, float b1, float b2, float eps,
                                                          float c1, float c2) {
  const uint64_t i = uint64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const int row = blockIdx.y;
  const int grp = row < 3 ? 0 : (row < 6 ? 1 : (row < 10 ? 2 : 3));
  const int first = grp == 0 ? 0 : (grp == 1 ? 3 : (grp == 2 ? 6 : 10));
  const uint64_t j = uint64_t(row - first) * n + i;
  const float gi = A.g[grp][j];
  float *m = A.m[grp], *v = A.v[grp], *p = A.p[grp];
  const float mi = b1 * m[j] + (1.f - b1) * gi;
  const float vi = b2 * v[j] + (1.f - b2) * gi * gi;
  m[j] = mi;
  v[j] = vi;
  const float mh = mi / c1;
  const float vh = vi / c2;
  float x = p[j] - A.lr[grp] * mh / (sqrtf(vh) + eps);
  if (grp == 3) x = fmaxf(x, 0.f);
  p[j] = x;
}

}  // namespace
}  // namespace fgs

using namespace fgs;

extern "C" int fgs_recon_step(fgs_gaussians_out *params, fgs_gaussian_grads *m, fgs_gaussian_grads *v,
                              fgs_gaussian_grads *grad, int64_t n, const fgs_geom *geom, int32_t view,
                              const float *gt, const fgs_grid *crop, const fgs_opts *opts,
                              const fgs_step_params *sp, const fgs_step_buffers *buf, fgs_workspace *ws_proj,
                              fgs_workspace *ws_crop, fgs_workspace *ws_loss, void *stream) {
  if (!params || !m || !v || !grad || !geom || !gt || !opts || !sp || !buf || !ws_proj || !ws_loss)
    return fail(FGS_E_INVALID, "null argument");
  if (!params->mean || !params->log_scale || !params->quat || !params->density || !m->mean || !m->log_scale ||
      !m->quat || !m->density || !v->mean || !v->log_scale || !v->quat || !v->density || !grad->mean ||
      !grad->log_scale || !grad->quat || !grad->density)
    return fail(FGS_E_INVALID, "null parameter, moment or gradient array");
  if (n <= 0 || view < 0 || view >= geom->n_views || sp->step < 1) return fail(FGS_E_INVALID, "n, view or step");
  if (!buf->img || !buf->grad_img || !buf->loss) return fail(FGS_E_INVALID, "null image buffers");
  const bool tv = crop && sp->tv_weight > 0.f;
  if (tv && (!ws_crop || !buf->crop_vol || !buf->crop_grad)) return fail(FGS_E_INVALID, "crop without buffers");
  if (opts->events) return fail(FGS_E_INVALID, "timing events are not taken by the step");
  hipStream_t s = static_cast<hipStream_t>(stream);
  const fgs_gaussians g{n, params->mean, params->log_scale, params->quat, params->density};
  const int64_t n_pix = int64_t(geom->det_w) * int64_t(geom->det_h);

  // 1. forward of the view, 2. the loss of Eq. 5 and its gradient image
  fgs_opts of = *opts;
  of.recompute = 1;
  of.accumulate = 0;
  int st = fgs_project_views_fwd(&g, geom, view, 1, &of, buf->img, ws_proj, stream);
  if (st != FGS_OK) return st;
  st = fgs_l1_loss_grad(buf->img, gt, n_pix, 1, buf->loss, buf->grad_img, ws_loss, stream);
  if (st != FGS_OK) return st;
  if (sp->ssim_weight > 0.f) {
    st = fgs_ssim_loss_grad(buf->img, gt, geom->det_w, geom->det_h, 1, sp->ssim_c1, sp->ssim_c2, sp->ssim_weight,
                            buf->loss + 1, buf->grad_img, 1, ws_loss, stream);
    if (st != FGS_OK) return st;
  }
  // 3. backward over the forward's lists
  fgs_opts ob = of;
  ob.recompute = 0;
  st = fgs_project_views_bwd(&g, geom, view, 1, &ob, buf->grad_img, grad, ws_proj, stream);
  if (st != FGS_OK) return st;
  // 4. the crop's TV prior, its gradient added to the rasterizer's
  if (tv) {
    fgs_opts ov{};
    ov.kappa = opts->kappa;
    ov.near_plane = opts->near_plane;
    ov.recompute = 1;
    st = fgs_voxelize_fwd(&g, crop, &ov, buf->crop_vol, ws_crop, stream);
    if (st != FGS_OK) return st;
    st = fgs_tv_loss_grad(buf->crop_vol, crop->dims, sp->tv_weight, buf->loss + 2, buf->crop_grad, ws_loss, stream);
    if (st != FGS_OK) return st;
    ov.recompute = 0;
    ov.accumulate = 1;
    st = fgs_voxelize_bwd(&g, crop, &ov, buf->crop_grad, grad, ws_crop, stream);
    if (st != FGS_OK) return st;
  }
  // 5. Adam on all parameters, one launch
  AdamGroups A;
  float *P[4] = {params->mean, params->log_scale, params->quat, params->density};
  const float *G[4] = {grad->mean, grad->log_scale, grad->quat, grad->density};
  float *M[4] = {m->mean, m->log_scale, m->quat, m->density};
  float *V[4] = {v->mean, v->log_scale, v->quat, v->density};
  for (int k = 0; k < 4; ++k) {
    A.p[k] = P[k];
    A.g[k] = G[k];
    A.m[k] = M[k];
    A.v[k] = V[k];
    A.lr[k] = sp->lr[k];
  }
  const float c1 = float(1.0 - std::pow(double(sp->beta1), double(sp->step)));
  const float c2 = float(1.0 - std::pow(double(sp->beta2), double(sp->step)));
  adam_groups_kernel<<<dim3(grid_for(uint64_t(n), 256), 11), 256, 0, s>>>(A, uint64_t(n), sp->beta1, sp->beta2,
                                                                          sp->eps, c1, c2);
  FGS_LAUNCH_CHECK("adam_groups_kernel");
  return FGS_OK;
}
