// fgs_recon_step: one optimiser step of the reconstruction loop (Sec. 3.4),
// the paper's unit of work, composed natively so that a step costs one call
// from the host instead of about twenty:
//   rasterizer forward of one view -> L1 (+ SSIM) of Eq. 5 against the
//   measured view, gradient image -> rasterizer backward (lists reused) ->
//   optionally a crop of the grid voxelized, its TV gradient and the
//   voxelizer backward added in -> one Adam launch over all 11 N parameters.
// The crop's voxelization, TV and voxelizer backward (into a gradient of
// its own) run on a second stream beside the view's forward and backward;
// Adam adds the two gradients.
// With key_capacity set in both rasterizer and crop workspaces nothing in the
// step waits for the GPU, so the host runs ahead.
//
// The values that change from step to step of one view (the crop's origin
// and Adam's bias corrections) are written by one small kernel into a device
// block (fgs_step_buffers.params) that the rest of the step reads. The rest
// can therefore be captured once per view in HIP graphs (fgs_step_graph_capture:
// the crop branch and the view branch, one graph each, and the Adam launch's
// arguments) and replayed for every later step of that view
// (fgs_step_graph_launch, the crop branch again on the second stream): the
// replay runs the same kernels on the same values as the direct call, and
// saves the per-kernel launch cost.
#include <algorithm>
#include <cmath>
#include <mutex>
#include <new>

#include "fgs_internal.h"

namespace fgs {
namespace {

// The step's per-call values, in the device block: crop origin (3), Adam's
// bias corrections 1 - beta1^t and 1 - beta2^t (2), three spare words.
constexpr int kStepParams = 8;
struct StepVals {
  float v[kStepParams];
};

__global__ void set_step_params_kernel(float *__restrict__ blk, StepVals s) {
  if (threadIdx.x < kStepParams) blk[threadIdx.x] = s.v[threadIdx.x];
}

// Adam (with bias correction) on the four parameter groups in one launch:
// blockIdx.y is the parameter row (3 mean, 3 log-scale, 4 quaternion, 1
// density rows of n values); density is clamped at zero. The arithmetic is
// that of fgs_adam_step, so the result is the same bit for bit. The bias
// corrections are read from the step block.
// g2 (may be null): a second gradient, added to g (g + g2, written back to
// g: the step's gradient) before the update.
struct AdamGroups {
  float *p[4];
  float *g[4];
  const float *g2[4];
  float *m[4], *v[4];
  float lr[4];
};

// The loss terms of the step (L1, SSIM, TV): out[k] = scale[k] * the sum of
// part[k]'s nb[k] per-block partial sums, for the terms with a non-null part.
struct LossFinish {
  const float *part[3];
  int nb[3];
  float scale[3];
  float *out;
};

// Blocks (x, 0..10) run Adam; in the extra row, block k < 3 adds up loss
// term k (their values are for reporting; nothing in the step reads them).
constexpr int kAdamRows = 11;

__global__ __launch_bounds__(256) void adam_groups_kernel(AdamGroups A, uint64_t n, float b1, float b2, float eps,
                                                          const float *__restrict__ blk, LossFinish F) {
  if (blockIdx.y == kAdamRows) {
    const int k = int(blockIdx.x);
    if (k >= 3 || !F.part[k]) return;
    __shared__ float sh[256 / 64];
    CompSum acc;
    for (int i = threadIdx.x; i < F.nb[k]; i += 256) acc.add(F.part[k][i]);
    const float t = block_sum_f32<256>(acc.value(), sh);
    if (threadIdx.x == 0) F.out[k] = F.scale[k] * t;
    return;
  }
  const uint64_t i = uint64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const float c1 = blk[3], c2 = blk[4];
  const int row = blockIdx.y;
  const int grp = row < 3 ? 0 : (row < 6 ? 1 : (row < 10 ? 2 : 3));
  const int first = grp == 0 ? 0 : (grp == 1 ? 3 : (grp == 2 ? 6 : 10));
  const uint64_t j = uint64_t(row - first) * n + i;
  float gi = A.g[grp][j];
  if (A.g2[grp]) {
    gi = gi + A.g2[grp][j];
    A.g[grp][j] = gi;
  }
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

struct StepArgs {
  fgs_gaussians_out *params;
  fgs_gaussian_grads *m, *v, *grad;
  int64_t n;
  const fgs_geom *geom;
  int32_t view;
  const float *gt;
  const fgs_grid *crop;
  const fgs_opts *opts;
  const fgs_step_params *sp;
  const fgs_step_buffers *buf;
  fgs_workspace *ws_proj, *ws_crop, *ws_loss;
};

// The loss workspace of a step, in floats: the SSIM term's partial sums
// (one per 16 x 16 tile), the L1 term's (per tile with SSIM, else per
// reduction block), the TV term's, the SSIM gradient's three maps, and the
// crop branch's parameter gradient.
struct LossParts {
  uint64_t ssim, l1, tv, gmaps, cgrad, total, n_tiles;
};

LossParts loss_parts(const StepArgs &a) {
  LossParts P{};
  const uint64_t n_pix = uint64_t(a.geom->det_w) * uint64_t(a.geom->det_h);
  P.n_tiles = ssim_tiles(a.geom->det_w, a.geom->det_h);
  auto up = [](uint64_t x) { return (x + 63) / 64 * 64; };  // 256-byte steps
  P.ssim = 0;
  P.l1 = up(P.n_tiles);
  P.tv = P.l1 + up(std::max<uint64_t>(P.n_tiles, kLossBlocks));
  P.gmaps = P.tv + up(kLossBlocks);
  // then, with a crop, the crop branch's parameter gradient (11 n floats)
  P.cgrad = P.gmaps + up(a.sp->ssim_weight > 0.f ? 3 * n_pix : 0);
  P.total = P.cgrad + (a.crop && a.sp->tv_weight > 0.f ? 11 * uint64_t(a.n) : 0);
  return P;
}

int check_args(const StepArgs &a) {
  if (!a.params || !a.m || !a.v || !a.grad || !a.geom || !a.gt || !a.opts || !a.sp || !a.buf || !a.ws_proj ||
      !a.ws_loss)
    return fail(FGS_E_INVALID, "null argument");
  const fgs_gaussians_out *P = a.params;
  if (!P->mean || !P->log_scale || !P->quat || !P->density || !a.m->mean || !a.m->log_scale || !a.m->quat ||
      !a.m->density || !a.v->mean || !a.v->log_scale || !a.v->quat || !a.v->density || !a.grad->mean ||
      !a.grad->log_scale || !a.grad->quat || !a.grad->density)
    return fail(FGS_E_INVALID, "null parameter, moment or gradient array");
  if (a.n <= 0 || a.view < 0 || a.view >= a.geom->n_views || a.sp->step < 1)
    return fail(FGS_E_INVALID, "n, view or step");
  if (!a.buf->img || !a.buf->grad_img || !a.buf->loss || !a.buf->params)
    return fail(FGS_E_INVALID, "null image, loss or step-parameter buffer");
  const bool tv = a.crop && a.sp->tv_weight > 0.f;
  if (tv && (!a.ws_crop || !a.buf->crop_vol || !a.buf->crop_grad))
    return fail(FGS_E_INVALID, "crop without buffers");
  if (a.opts->events) return fail(FGS_E_INVALID, "timing events are not taken by the step");
  if (a.geom->det_w <= 0 || a.geom->det_h <= 0) return fail(FGS_E_INVALID, "detector size");
  const LossParts LP = loss_parts(a);
  a.ws_loss->needed = LP.total * sizeof(float);
  if (!a.ws_loss->ptr || a.ws_loss->bytes < a.ws_loss->needed)
    return fail(FGS_E_CAPACITY, "loss workspace too small");
  a.ws_loss->kind = 0;
  return FGS_OK;
}

StepVals step_vals(const StepArgs &a) {
  StepVals s{};
  const bool tv = a.crop && a.sp->tv_weight > 0.f;
  for (int k = 0; k < 3; ++k) s.v[k] = tv ? a.crop->origin[k] : 0.f;
  s.v[3] = float(1.0 - std::pow(double(a.sp->beta1), double(a.sp->step)));
  s.v[4] = float(1.0 - std::pow(double(a.sp->beta2), double(a.sp->step)));
  return s;
}

// The crop branch of a step (its binning, voxelization, TV and voxelizer
// backward into a gradient of its own) depends on nothing the view's
// forward and backward compute, so it runs on a second stream: forked from
// the step's stream once the step block is written, joined before Adam adds
// its gradient to the view's. Its kernels are small and latency-bound, so
// they overlap with the view's.
struct Side {
  hipStream_t s = nullptr;
  hipEvent_t fork = nullptr, join = nullptr;
};

int side_create(Side &x) {
  if (!x.s) FGS_HIP(hipStreamCreateWithFlags(&x.s, hipStreamNonBlocking));
  if (!x.fork) FGS_HIP(hipEventCreateWithFlags(&x.fork, hipEventDisableTiming));
  if (!x.join) FGS_HIP(hipEventCreateWithFlags(&x.join, hipEventDisableTiming));
  return FGS_OK;
}

// The loss terms' sums the Adam launch finishes (positions from the
// arguments alone).
LossFinish loss_finish(const StepArgs &a) {
  const LossParts LP = loss_parts(a);
  float *lp = static_cast<float *>(a.ws_loss->ptr);
  const fgs_step_params *sp = a.sp;
  const int64_t n_pix = int64_t(a.geom->det_w) * int64_t(a.geom->det_h);
  LossFinish F{};
  F.out = a.buf->loss;
  F.part[0] = lp + LP.l1;
  F.scale[0] = float(1.0 / double(n_pix));
  if (sp->ssim_weight > 0.f) {
    F.nb[0] = int(LP.n_tiles);
    F.part[1] = lp + LP.ssim;
    F.nb[1] = int(LP.n_tiles);
    F.scale[1] = float(double(sp->ssim_weight) / double(n_pix));
  } else {
    F.nb[0] = loss_blocks(uint64_t(n_pix));
  }
  if (a.crop && sp->tv_weight > 0.f) {
    const uint64_t nc = uint64_t(a.crop->dims[0]) * a.crop->dims[1] * a.crop->dims[2];
    F.part[2] = lp + LP.tv;
    F.nb[2] = loss_blocks(nc);
    F.scale[2] = float(double(sp->tv_weight) / double(nc));
  }
  return F;
}

fgs_opts crop_opts(const StepArgs &a, int recompute, int accumulate) {
  fgs_opts ov{};
  ov.kappa = a.opts->kappa;
  ov.near_plane = a.opts->near_plane;
  ov.recompute = recompute;
  ov.accumulate = accumulate;
  return ov;
}

fgs_gaussians gauss(const StepArgs &a) {
  return fgs_gaussians{a.n, a.params->mean, a.params->log_scale, a.params->quat, a.params->density};
}

// The crop branch's parameter gradient, in the loss workspace.
fgs_gaussian_grads crop_param_grad(const StepArgs &a) {
  float *c = static_cast<float *>(a.ws_loss->ptr) + loss_parts(a).cgrad;
  const uint64_t n = uint64_t(a.n);
  return fgs_gaussian_grads{c, c + 3 * n, c + 6 * n, c + 10 * n};
}

// The crop branch: the crop voxelized at the block's origin, the TV term's
// gradient and partial sums (the TV prior of Eq. 5), and the voxelizer
// backward of that gradient into the branch's own parameter gradient (the
// Adam launch adds it to the view's).
int crop_branch(const StepArgs &a, hipStream_t sc) {
  const fgs_gaussians g = gauss(a);
  const fgs_opts ov = crop_opts(a, 1, 0);
  int st = vox_forward(&g, a.crop, &ov, a.buf->crop_vol, a.ws_crop, sc, a.buf->params);
  if (st != FGS_OK) return st;
  const LossParts LP = loss_parts(a);
  float *lp = static_cast<float *>(a.ws_loss->ptr);
  st = tv_partials(a.buf->crop_vol, a.crop->dims, a.sp->tv_weight, a.buf->crop_grad, lp + LP.tv, sc);
  if (st != FGS_OK) return st;
  const fgs_opts ob = crop_opts(a, 0, 0);
  fgs_gaussian_grads cg = crop_param_grad(a);
  return vox_backward(&g, a.crop, &ob, a.buf->crop_grad, &cg, a.ws_crop, sc, a.buf->params);
}

// The view branch: forward of the view, the loss of Eq. 5 (the L1 term's
// gradient sign(x - y) / n_pix, with the SSIM term's added in the same
// kernel; the terms' partial sums wait for the Adam launch), backward over
// the forward's lists (writing the gradient).
int view_branch(const StepArgs &a, hipStream_t s) {
  void *stream = static_cast<void *>(s);
  const fgs_step_params *sp = a.sp;
  const fgs_step_buffers *buf = a.buf;
  const fgs_gaussians g = gauss(a);
  const int64_t n_pix = int64_t(a.geom->det_w) * int64_t(a.geom->det_h);
  const LossParts LP = loss_parts(a);
  float *lp = static_cast<float *>(a.ws_loss->ptr);
  fgs_opts of = *a.opts;
  of.recompute = 1;
  of.accumulate = 0;
  int st = fgs_project_views_fwd(&g, a.geom, a.view, 1, &of, buf->img, a.ws_proj, stream);
  if (st != FGS_OK) return st;
  const float inv_p = 1.f / float(n_pix);
  if (sp->ssim_weight > 0.f)
    st = ssim_l1_partials(buf->img, a.gt, a.geom->det_w, a.geom->det_h, sp->ssim_c1, sp->ssim_c2, sp->ssim_weight,
                          inv_p, buf->grad_img, lp + LP.gmaps, lp + LP.ssim, lp + LP.l1, s);
  else
    st = l1_partials(buf->img, a.gt, uint64_t(n_pix), inv_p, buf->grad_img, lp + LP.l1, s);
  if (st != FGS_OK) return st;
  fgs_opts ob = of;
  ob.recompute = 0;
  return fgs_project_views_bwd(&g, a.geom, a.view, 1, &ob, buf->grad_img, a.grad, a.ws_proj, stream);
}

// The tail (after both branches): Adam on all parameters in one launch,
// which adds the crop branch's gradient to the view's (the sum is the step's
// gradient, written to grad: the one fgs_voxelize_bwd accumulating onto
// the rasterizer's gives, bit for bit) and finishes the loss terms. Its
// arguments depend on the step's arguments only, so a captured step keeps
// them and launches the kernel itself.
struct TailArgs {
  AdamGroups A;
  LossFinish F;
  uint64_t n;
  float b1, b2, eps;
  const float *blk;
};

TailArgs tail_args(const StepArgs &a) {
  const fgs_step_params *sp = a.sp;
  const bool tv = a.crop && sp->tv_weight > 0.f;
  const fgs_gaussian_grads cg = tv ? crop_param_grad(a) : fgs_gaussian_grads{};
  TailArgs t{};
  float *P[4] = {a.params->mean, a.params->log_scale, a.params->quat, a.params->density};
  float *G[4] = {a.grad->mean, a.grad->log_scale, a.grad->quat, a.grad->density};
  const float *G2[4] = {cg.mean, cg.log_scale, cg.quat, cg.density};
  float *M[4] = {a.m->mean, a.m->log_scale, a.m->quat, a.m->density};
  float *V[4] = {a.v->mean, a.v->log_scale, a.v->quat, a.v->density};
  for (int k = 0; k < 4; ++k) {
    t.A.p[k] = P[k];
    t.A.g[k] = G[k];
    t.A.g2[k] = G2[k];
    t.A.m[k] = M[k];
    t.A.v[k] = V[k];
    t.A.lr[k] = sp->lr[k];
  }
  t.F = loss_finish(a);
  t.n = uint64_t(a.n);
  t.b1 = sp->beta1;
  t.b2 = sp->beta2;
  t.eps = sp->eps;
  t.blk = a.buf->params;
  return t;
}

int launch_tail(const TailArgs &t, hipStream_t s) {
  adam_groups_kernel<<<dim3(std::max(grid_for(t.n, 256), 3u), kAdamRows + 1), 256, 0, s>>>(t.A, t.n, t.b1, t.b2,
                                                                                           t.eps, t.blk, t.F);
  FGS_LAUNCH_CHECK("adam_groups_kernel");
  return FGS_OK;
}

int tail(const StepArgs &a, hipStream_t s) { return launch_tail(tail_args(a), s); }

// Makes s wait for the crop branch when the step returns early (an error,
// e.g. a workspace to grow) after forking it.
struct JoinOnExit {
  hipStream_t s;
  const Side *side = nullptr;
  ~JoinOnExit() {
    if (side) (void)hipStreamWaitEvent(s, side->join, 0);
  }
};

// Everything after the step block is written (it reads the crop origin and
// the bias corrections from buf->params). side (may be null): the crop
// branch's stream and events, else the crop runs in line on s.
int step_body(const StepArgs &a, hipStream_t s, const Side *side) {
  const bool tv = a.crop && a.sp->tv_weight > 0.f;
  JoinOnExit join_on_exit{s};
  if (tv) {
    hipStream_t sc = s;
    if (side) {
      FGS_HIP(hipEventRecord(side->fork, s));
      FGS_HIP(hipStreamWaitEvent(side->s, side->fork, 0));
      sc = side->s;
    }
    const int st = crop_branch(a, sc);
    if (side) {
      FGS_HIP(hipEventRecord(side->join, side->s));
      join_on_exit.side = side;  // until the tail waits for it
    }
    if (st != FGS_OK) return st;
  }
  int st = view_branch(a, s);
  if (st != FGS_OK) return st;
  if (tv && side) {
    join_on_exit.side = nullptr;
    FGS_HIP(hipStreamWaitEvent(s, side->join, 0));
  }
  return tail(a, s);
}

// Direct steps share one side stream per device; the lock covers a step's
// enqueueing, so the fork and join events of concurrent callers do not mix.
constexpr int kMaxDevices = 64;
std::mutex g_side_mu;
Side g_side[kMaxDevices];

int set_params(float *blk, const StepVals &v, hipStream_t s) {
  set_step_params_kernel<<<1, 64, 0, s>>>(blk, v);
  FGS_LAUNCH_CHECK("set_step_params_kernel");
  return FGS_OK;
}

}  // namespace
}  // namespace fgs

using namespace fgs;

// A captured step of one view: the instantiated graphs of its crop branch
// (null without a crop) and its view branch, the tail's kernel arguments,
// and what a launch must match. A launch runs the crop branch on the side stream beside the
// view branch, as a direct step does.
struct fgs_step_graph {
  hipGraphExec_t crop;
  hipGraphExec_t view_branch;
  fgs::TailArgs tail;
  float *params;
  int32_t view;
  int32_t crop_dims[3];
  int has_crop;
};

namespace {

// Records fn(stream) into an instantiated graph, on a private stream.
template <typename Fn>
int capture(Fn &&fn, hipGraphExec_t *out) {
  *out = nullptr;
  hipStream_t cs;
  hipError_t e = hipStreamCreateWithFlags(&cs, hipStreamNonBlocking);
  if (e != hipSuccess) return hip_fail(e, "hipStreamCreateWithFlags");
  e = hipStreamBeginCapture(cs, hipStreamCaptureModeThreadLocal);
  if (e != hipSuccess) {
    (void)hipStreamDestroy(cs);
    return hip_fail(e, "hipStreamBeginCapture");
  }
  const int st = fn(cs);
  hipGraph_t graph = nullptr;
  e = hipStreamEndCapture(cs, &graph);
  (void)hipStreamDestroy(cs);
  if (st != FGS_OK || e != hipSuccess) {
    if (graph) (void)hipGraphDestroy(graph);
    // a capture cut short leaves its error as the runtime's last error,
    // which the next launch check would report
    (void)hipGetLastError();
    return st != FGS_OK ? st : hip_fail(e, "hipStreamEndCapture");
  }
  e = hipGraphInstantiate(out, graph, nullptr, nullptr, 0);
  (void)hipGraphDestroy(graph);
  if (e != hipSuccess) {
    *out = nullptr;
    return hip_fail(e, "hipGraphInstantiate");
  }
  return FGS_OK;
}

void destroy_execs(fgs_step_graph &g) {
  if (g.crop) (void)hipGraphExecDestroy(g.crop);
  if (g.view_branch) (void)hipGraphExecDestroy(g.view_branch);
  g.crop = g.view_branch = nullptr;
}

// The calling device's shared side stream, created on first use; the
// caller holds g_side_mu.
int device_side(Side **out) {
  int dev = -1;
  FGS_HIP(hipGetDevice(&dev));
  if (dev < 0 || dev >= kMaxDevices) return fail(FGS_E_UNSUPPORTED, "device ordinal beyond 63");
  const int st = side_create(g_side[dev]);
  if (st != FGS_OK) return st;
  *out = &g_side[dev];
  return FGS_OK;
}

}  // namespace

extern "C" int fgs_recon_step(fgs_gaussians_out *params, fgs_gaussian_grads *m, fgs_gaussian_grads *v,
                              fgs_gaussian_grads *grad, int64_t n, const fgs_geom *geom, int32_t view,
                              const float *gt, const fgs_grid *crop, const fgs_opts *opts,
                              const fgs_step_params *sp, const fgs_step_buffers *buf, fgs_workspace *ws_proj,
                              fgs_workspace *ws_crop, fgs_workspace *ws_loss, void *stream) {
  const StepArgs a{params, m, v, grad, n, geom, view, gt, crop, opts, sp, buf, ws_proj, ws_crop, ws_loss};
  int st = check_args(a);
  if (st != FGS_OK) return st;
  hipStream_t s = static_cast<hipStream_t>(stream);
  const bool tv = crop && sp->tv_weight > 0.f;
  std::unique_lock<std::mutex> lock(g_side_mu, std::defer_lock);
  Side *side = nullptr;
  if (tv) {
    lock.lock();
    st = device_side(&side);
    if (st != FGS_OK) return st;
  }
  st = set_params(buf->params, step_vals(a), s);
  if (st != FGS_OK) return st;
  return step_body(a, s, side);
}

extern "C" int fgs_step_graph_capture(fgs_gaussians_out *params, fgs_gaussian_grads *m, fgs_gaussian_grads *v,
                                      fgs_gaussian_grads *grad, int64_t n, const fgs_geom *geom, int32_t view,
                                      const float *gt, const fgs_grid *crop, const fgs_opts *opts,
                                      const fgs_step_params *sp, const fgs_step_buffers *buf,
                                      fgs_workspace *ws_proj, fgs_workspace *ws_crop, fgs_workspace *ws_loss,
                                      fgs_step_graph **out) {
  if (!out) return fail(FGS_E_INVALID, "null output");
  *out = nullptr;
  const StepArgs a{params, m, v, grad, n, geom, view, gt, crop, opts, sp, buf, ws_proj, ws_crop, ws_loss};
  int st = check_args(a);
  if (st != FGS_OK) return st;
  const bool tv = crop && sp->tv_weight > 0.f;
  // a captured step may not wait for the GPU: both list sets need a fixed capacity
  if (ws_proj->key_capacity == 0 || (tv && ws_crop->key_capacity == 0))
    return fail(FGS_E_INVALID, "graph capture needs key_capacity set in the rasterizer and crop workspaces");
  fgs_step_graph G{};
  if (tv) st = capture([&](hipStream_t cs) { return crop_branch(a, cs); }, &G.crop);
  if (st == FGS_OK) st = capture([&](hipStream_t cs) { return view_branch(a, cs); }, &G.view_branch);
  G.tail = tail_args(a);
  if (st != FGS_OK) {
    destroy_execs(G);
    return st;
  }
  fgs_step_graph *gph = new (std::nothrow) fgs_step_graph(G);
  if (!gph) {
    destroy_execs(G);
    return fail(FGS_E_INVALID, "out of host memory");
  }
  gph->params = buf->params;
  gph->view = view;
  gph->has_crop = tv ? 1 : 0;
  for (int k = 0; k < 3; ++k) gph->crop_dims[k] = tv ? crop->dims[k] : 0;
  *out = gph;
  return FGS_OK;
}

extern "C" int fgs_step_graph_launch(fgs_step_graph *gph, const fgs_step_params *sp, const fgs_grid *crop,
                                     void *stream) {
  if (!gph || !sp) return fail(FGS_E_INVALID, "null argument");
  if (sp->step < 1) return fail(FGS_E_INVALID, "step must be >= 1");
  if (gph->has_crop) {
    if (!crop) return fail(FGS_E_INVALID, "the captured step has a crop: pass one");
    for (int k = 0; k < 3; ++k)
      if (crop->dims[k] != gph->crop_dims[k]) return fail(FGS_E_INVALID, "crop dims differ from the captured ones");
  }
  StepVals vals{};
  for (int k = 0; k < 3; ++k) vals.v[k] = gph->has_crop ? crop->origin[k] : 0.f;
  vals.v[3] = float(1.0 - std::pow(double(sp->beta1), double(sp->step)));
  vals.v[4] = float(1.0 - std::pow(double(sp->beta2), double(sp->step)));
  hipStream_t s = static_cast<hipStream_t>(stream);
  std::unique_lock<std::mutex> lock(g_side_mu, std::defer_lock);
  Side *side = nullptr;
  if (gph->has_crop) {
    lock.lock();
    const int st = device_side(&side);
    if (st != FGS_OK) return st;
  }
  int st = set_params(gph->params, vals, s);
  if (st != FGS_OK) return st;
  if (side) {
    FGS_HIP(hipEventRecord(side->fork, s));
    FGS_HIP(hipStreamWaitEvent(side->s, side->fork, 0));
    FGS_HIP(hipGraphLaunch(gph->crop, side->s));
    FGS_HIP(hipEventRecord(side->join, side->s));
  }
  const hipError_t e = hipGraphLaunch(gph->view_branch, s);
  if (side) FGS_HIP(hipStreamWaitEvent(s, side->join, 0));
  if (e != hipSuccess) return hip_fail(e, "hipGraphLaunch");
  return launch_tail(gph->tail, s);
}

extern "C" int fgs_step_graph_destroy(fgs_step_graph *gph) {
  if (!gph) return FGS_OK;
  hipError_t e = hipSuccess;
  for (hipGraphExec_t x : {gph->crop, gph->view_branch})
    if (x) {
      const hipError_t ex = hipGraphExecDestroy(x);
      if (e == hipSuccess) e = ex;
    }
  delete gph;
  if (e != hipSuccess) return hip_fail(e, "hipGraphExecDestroy");
  return FGS_OK;
}
