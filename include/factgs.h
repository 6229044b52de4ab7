/*
 * factgs.h -- C ABI of the MI355X (gfx950) Gaussian X-ray rasterizer and
 * voxelizer library (libfactgs.so).
 *
 * The library implements the two differentiable renderers of the FaCT-GS
 * CT-reconstruction method (arXiv 2604.01844):
 *
 *   - project_views: the X-ray rasterizer. Each 3D Gaussian (Eq. 1:
 *     density rho, mean p, covariance Sigma) is projected, per cone-beam (or
 *     parallel-beam) view, to a 2D Gaussian on the flat detector carrying the
 *     ray-integral density factor mu (Eq. 4, Sec. 3.2); every detector pixel
 *     is the order-free sum of the splats whose 3-sigma support contains it
 *     (Sec. 3.2 cutoff, Sec. 3.5 "no depth ordering").
 *   - voxelize: the density field sigma(x) = sum_i G_i(x) (Eq. 2) sampled at
 *     the centres of a regular grid, each Gaussian limited to its 3-sigma
 *     ellipsoid (Sec. 3.3).
 *
 * and, for each, the backward pass: the gradient of a scalar loss with
 * respect to the 11 parameters per Gaussian (Sec. 5: position 3, scale 3,
 * quaternion 4, density 1), given the loss gradient with respect to the
 * image or volume. Gradients are those of the function with its support
 * held fixed (the hard cutoff contributes no derivative).
 *
 * Conventions
 *   Gaussians: structure of arrays in device memory, float32:
 *     mean[3][n] (x, y, z rows), log_scale[3][n] (natural log of the
 *     standard deviation along each principal axis), quat[4][n] (w, x, y, z,
 *     any non-zero norm; normalised inside), density[n] (linear rho).
 *     Sigma = R(q/|q|) diag(exp(2 log_scale)) R^T.
 *   World: the reconstruction cube is [-1/2, 1/2]^3, rotation axis +z.
 *   View at angle th: source at sod (cos th, sin th, 0); camera rows
 *     e0 = (-sin th, cos th, 0), e1 = (0, 0, -1), e2 = (-cos th, -sin th, 0);
 *     the flat detector is at distance sdd from the source along e2.
 *     Detector pixel (j, i) (column j, row i) is sampled at continuous
 *     pixel coordinates (j + 1/2, i + 1/2); the principal ray hits
 *     (det_w/2 + off_u, det_h/2 + off_v). Images are [view][det_h][det_w].
 *   Support: a (pixel, Gaussian) pair contributes iff its Mahalanobis
 *     distance in the 2D splat satisfies d^2 <= kappa^2 (kappa = 3).
 *   Grids: voxel (ix, iy, iz) has its centre at origin + (index + 1/2) *
 *     spacing; volumes are [nz][ny][nx], x fastest.
 *
 * Ownership and asynchrony
 *   Every pointer argument named as device memory must be a device pointer
 *   on the current HIP device, 16-byte aligned. The caller owns all device
 *   memory: outputs and the workspace. The library never allocates device
 *   memory and keeps no state between calls except a thread-local error
 *   message. All work is enqueued on `stream` (a hipStream_t passed as
 *   void*; NULL = the default stream). Calls return without waiting for
 *   the GPU, except where a call must learn the number of (tile, Gaussian)
 *   pairs to size its workspace use: it then waits on `stream` for one
 *   4-byte device-to-host copy (documented per call).
 *
 * Errors
 *   Every entry point returns an fgs_status. No C++ exception crosses the
 *   ABI. On an error nothing is written to the outputs unless stated, and
 *   fgs_last_error() returns a thread-local description.
 */
#ifndef FACTGS_H
#define FACTGS_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
  FGS_OK = 0,
  FGS_E_INVALID = -1,     /* null pointer, non-positive size, kappa <= 0, view range out of bounds */
  FGS_E_CAPACITY = -2,    /* workspace too small: ws->needed holds the required bytes; retry */
  FGS_E_HIP = -3,         /* HIP launch or runtime error; see fgs_last_error() */
  FGS_E_UNSUPPORTED = -4  /* a size beyond what the kernels index (e.g. 2^32 pairs per call) */
} fgs_status;

enum { FGS_CONE = 0, FGS_PARALLEL = 1 };

/* Gaussian parameters (Eq. 1 and the 11-value parameterisation of Sec. 5). */
typedef struct {
  int64_t n;               /* number of Gaussians, >= 1 */
  const float *mean;       /* device [3][n] */
  const float *log_scale;  /* device [3][n] */
  const float *quat;       /* device [4][n], (w, x, y, z) */
  const float *density;    /* device [n] */
} fgs_gaussians;

/* Gradient outputs, same shapes as fgs_gaussians; overwritten, never accumulated. */
typedef struct {
  float *mean;       /* device [3][n] */
  float *log_scale;  /* device [3][n] */
  float *quat;       /* device [4][n] */
  float *density;    /* device [n] */
} fgs_gaussian_grads;

/* Gaussian parameters written by an initialiser: same layout as fgs_gaussians. */
typedef fgs_gaussian_grads fgs_gaussians_out;

/* Scanner geometry (Sec. 3.2: cone-beam pinhole model or parallel beam). */
typedef struct {
  int32_t mode;          /* FGS_CONE or FGS_PARALLEL */
  int32_t n_views;       /* number of entries in angles */
  const float *angles;   /* device [n_views], radians */
  float sod;             /* source-to-rotation-axis distance (cone) */
  float sdd;             /* source-to-detector distance (cone) */
  int32_t det_w, det_h;  /* detector pixels */
  float pitch_u, pitch_v;/* detector pixel pitch (world units at the detector) */
  float off_u, off_v;    /* principal-point offset in pixels */
} fgs_geom;

/* Regular voxel grid (any sub-box of space, e.g. a 32^3 crop). */
typedef struct {
  float origin[3];       /* outer corner of voxel (0, 0, 0) */
  float spacing[3];      /* voxel size per axis, > 0 */
  int32_t dims[3];       /* nx, ny, nz, >= 1 */
} fgs_grid;

typedef struct {
  float kappa;           /* support radius in standard deviations (3) */
  float near_plane;      /* cone beam: Gaussians with camera depth <= near are culled (1e-2) */
  int32_t recompute;     /* backward only: 1 = rebuild the per-tile lists; 0 = reuse those that
                            the forward call left in the same workspace (same inputs) */
  int32_t accumulate;    /* backward only: 1 = add the gradients to what `out` holds (summing
                            over view chunks or voxel slabs); 0 = overwrite */
  int32_t ablate;        /* rasterizer only: 0 = the library's design. For measuring what its
                            parts contribute (an analogue of the paper's Table 3), a bitmask of
                            FGS_ABLATE_* that switches parts off; results stay correct. Other
                            bits: FGS_E_INVALID */
  int32_t model;         /* rasterizer: FGS_MODEL_SPLAT (0) or FGS_MODEL_RAY_EXACT (1); other
                            values, or a non-zero value for the voxelizer: FGS_E_INVALID */
  void *events;          /* optional hipEvent_t[2] (NULL = none): recorded on the stream right
                            before and right after the call's pixel or voxel kernel (splat
                            forward/backward, voxel forward/backward), for timing that kernel */
  float density_aabb_tau;/* density-aware support (Sec. 3.5: the axis-aligned boxes also take
                            the density into account), in the units of the image (rasterizer) or
                            volume (voxelizer). 0 = off: the kappa support. tau > 0: a pair
                            is kept iff d^2 <= min(kappa^2, 2 ln(peak / tau)), i.e. also
                            its contribution peak exp(-d^2/2) is at least tau, with peak = w
                            = rho mu for a splat and rho for the voxelizer; the tile boxes
                            shrink to that support, and a Gaussian whose peak is <= tau is
                            left out. Negative or non-finite: FGS_E_INVALID. Splat model
                            without ablation switches only (FGS_E_UNSUPPORTED otherwise).
                            Gradients are those of the function with this support held
                            fixed, as for kappa. */
} fgs_opts;

/* Tile sizes are fixed: 16 x 16 pixels for the rasterizer (four 8 x 8
 * quadrants culled separately inside each) and 8 x 8 x 8 voxels for the
 * voxelizer. The kernels' lane layouts are built around them. */

/* fgs_opts.model (rasterizer).
 * FGS_MODEL_SPLAT: the method's splat M (Eq. 4): per (view, Gaussian) a 2D
 *   Gaussian on the detector with the integration factor mu, kept where its
 *   Mahalanobis distance d <= kappa.
 * FGS_MODEL_RAY_EXACT: the exact line integral E of Eq. 3 per ray, kept where
 *   the ray passes within Mahalanobis distance kappa of the mean (the
 *   support is the detector image of the kappa-ellipsoid). In cone beam a
 *   Gaussian is also left out of a view when the source lies inside its
 *   kappa-ellipsoid. About 2.5-3.5x the pixel work of the splat. In parallel
 *   beam the two models coincide and the splat kernels run. The ablation
 *   switches apply to the splat model only (FGS_E_UNSUPPORTED otherwise). */
#define FGS_MODEL_SPLAT 0
#define FGS_MODEL_RAY_EXACT 1

/* fgs_opts.ablate bits (rasterizer). */
#define FGS_ABLATE_SQUARE_BOX 1     /* tile rectangles from the square of half-side kappa sqrt(lambda_max)
                                       (the circle bound of the original splatting) instead of the
                                       support ellipse's exact box */
#define FGS_ABLATE_QUADRANT_CULL 2  /* no per-quadrant culling inside a tile: every pixel of every
                                       listed (tile, Gaussian) pair is evaluated */
#define FGS_ABLATE_PER_PIXEL_BWD 4  /* pixel-parallel backward: per listed Gaussian, the tile's pixel
                                       contributions are summed across the wave and added to the
                                       record with float atomics (not deterministic) instead of the
                                       per-Gaussian pair slots */

/* Caller-owned device workspace. The "out" fields describe what the last
 * forward call left in it; a backward call with opts.recompute = 0 reads
 * them, so pass the same struct back unchanged. */
typedef struct {
  void *ptr;             /* device memory, 256-byte aligned */
  uint64_t bytes;        /* size of ptr */
  uint64_t needed;       /* out: bytes this call needs (on FGS_OK and FGS_E_CAPACITY) */
  uint64_t n_pairs;      /* out: (tile, Gaussian) pairs of the last binning */
  uint64_t n_records;    /* out: records of the last binning */
  uint64_t n_tiles;      /* out: tiles of the last binning */
  int32_t kind;          /* out: 0 none, 1 rasterizer lists (splat model), 2 voxelizer lists,
                            3 rasterizer lists (ray-exact model) */
  int32_t tile_bits;     /* out: rasterizer: width of the tile field of its keys */
  uint64_t key_capacity; /* in: 0 = the rasterizer and voxelizer calls read the number of
                            (tile, Gaussian) pairs back and size the lists by it (one wait on
                            the stream per call). > 0 (below 2^32) = they lay the lists out for
                            at most this many pairs and keep the count on the device: no wait,
                            so a sequence of calls can be captured in a HIP graph. ws->needed
                            and ws->n_pairs then describe the capacity (the call returns
                            FGS_E_CAPACITY before any GPU work if bytes is too small for it).
                            A call whose pairs exceed it bins nothing (its image or volume is
                            zero, its gradient contribution zero) and reports that through
                            `overflow`. A backward that reuses the lists must see the same
                            capacity. */
  uint32_t *overflow;    /* in, used with key_capacity > 0 (may be NULL): device uint32[2] that
                            the caller zeroes; a call that overflows sets overflow[0] = 1 and
                            raises overflow[1] to the pairs it needed (at most 2^32 - 1). Never
                            cleared by the library. */
  int32_t record_bits;   /* out: rasterizer: 0 = key/value lists (key = view << tile_bits | tile,
                            value = record); > 0 = one-word lists, each word tile << record_bits
                            | record (used when the tile field and the record index fit 32 bits:
                            half the sort's bytes), the view being record / n_gauss */
  uint64_t n_gauss;      /* out: rasterizer: Gaussians of the last binning (records = views x
                            n_gauss) */
} fgs_workspace;

/* Additive ellipsoid phantom: sum_e amp_e * [x inside ellipsoid e]. Used to
 * make synthetic ground truth (stands in for the paper's datasets). */
typedef struct {
  int64_t n;             /* ellipsoids */
  const double *centre;  /* device [n][3] */
  const double *semi;    /* device [n][3] semi-axes */
  const double *quat;    /* device [n][4] (w, x, y, z), any non-zero norm */
  const double *amp;     /* device [n] */
} fgs_phantom;

/* ---------------------------------------------------------------------
 * X-ray rasterizer (Eq. 3-4, Sec. 3.2, Sec. 3.5).
 * Renders views [view_begin, view_begin + view_count) into
 * img[view_count][det_h][det_w] (device, overwritten), with the model
 * opts.model selects (the splat M of Eq. 4, or the ray-exact E of Eq. 3).
 * Pipeline: per-(view, Gaussian) splat records; tile counts, exclusive scan
 * and key emission (keys = view * tiles_per_view + tile, row-major inside
 * each record's axis-aligned tile rectangle); stable LSD radix sort; per-tile
 * ranges; per-tile splat. Per pixel the sum runs over its tile's list (in
 * ascending Gaussian index after the stable sort) in an order fixed by the
 * list and the launch shape alone: each 8-lane half of a quadrant group
 * takes alternate entries, the interior variant takes a batch's interior
 * pairs first, a few-tile call sums its work units' partials in unit order.
 * No atomics: deterministic and bit-reproducible for a given call shape.
 * Synchronisation: waits on `stream` once to read the pair count, unless
 * ws->key_capacity > 0 (then not at all).
 * Workspace: if ws->bytes < ws->needed the call returns FGS_E_CAPACITY with
 * ws->needed set and no output written; grow and retry. The workspace then
 * holds the lists the backward can reuse (opts.recompute = 0).
 * ------------------------------------------------------------------- */
int fgs_project_views_fwd(const fgs_gaussians *g, const fgs_geom *geom, int32_t view_begin,
                          int32_t view_count, const fgs_opts *opts, float *img,
                          fgs_workspace *ws, void *stream);

/* For callers that cannot allocate device memory or hand over a workspace
 * (code under HIP graph capture, tight serving loops, harnesses that forbid
 * hipMalloc): fgs_project_views_fwd with the same arguments and results,
 * minus the workspace. The lists, records and partial images live in a
 * fixed 64 MiB device array inside the library, one per GPU, held from the
 * first call on that GPU until the process ends; the call allocates nothing
 * (no hipMalloc, no allocating library routine). 64 MiB holds one 512 x 512
 * view of about 50,000 Gaussians; a call that needs more returns
 * FGS_E_CAPACITY (the message names the bytes needed) before writing img,
 * and cannot be retried with more room: split the views or use
 * fgs_project_views_fwd. Every call on a GPU uses that GPU's one array:
 * calls that overlap on one GPU (other streams, other host threads) race
 * and must be serialised by the caller. No lists are left for a backward.
 * Synchronisation: as fgs_project_views_fwd (one wait for the pair count). */
int fgs_project_views_fwd_noalloc(const fgs_gaussians *g, const fgs_geom *geom, int32_t view_begin,
                                  int32_t view_count, const fgs_opts *opts, float *img, void *stream);

/* Backward of fgs_project_views_fwd: given grad_img[view_count][det_h][det_w]
 * (device) = dL/dimg, writes dL/d(mean, log_scale, quat, density) summed
 * over the views (overwritten). Per (tile, Gaussian) pair the pixel sums
 * are formed by one lane (no atomics), then reduced per (view, Gaussian) in
 * list order and per Gaussian in view order: deterministic.
 * opts.recompute = 1 rebuilds the lists (and may return FGS_E_CAPACITY like
 * the forward); 0 requires the workspace the forward call filled. */
int fgs_project_views_bwd(const fgs_gaussians *g, const fgs_geom *geom, int32_t view_begin,
                          int32_t view_count, const fgs_opts *opts, const float *grad_img,
                          fgs_gaussian_grads *out, fgs_workspace *ws, void *stream);

/* ---------------------------------------------------------------------
 * One optimiser step of the reconstruction loop (Sec. 3.4: one view per
 * step, the loss of Eq. 5), composed in the library so that a step is one
 * host call.
 * ------------------------------------------------------------------- */
typedef struct {
  float ssim_weight;     /* weight of the SSIM term of Eq. 5 (0 = L1 only) */
  float ssim_c1, ssim_c2;/* SSIM constants (0.01^2, 0.03^2 for unit dynamic range) */
  float tv_weight;       /* weight of the crop's TV term (0 = none) */
  float lr[4];           /* Adam learning rates: mean, log-scale, quaternion, density */
  float beta1, beta2, eps;
  int32_t step;          /* Adam step count of this step (>= 1): bias correction */
} fgs_step_params;

typedef struct {
  float *img;            /* device [det_h][det_w]: the rendered view (overwritten) */
  float *grad_img;       /* device [det_h][det_w]: dL/dimg (overwritten) */
  float *crop_vol;       /* device crop voxels (with a crop): its voxelization */
  float *crop_grad;      /* device crop voxels (with a crop): dTV/dvol */
  float *loss;           /* device [3]: L1 term, SSIM term (with ssim_weight > 0), TV term (with
                            a crop); entries of absent terms are left as they are */
  float *params;         /* device [8], caller-owned: the step's per-call values (crop origin,
                            Adam's bias corrections), written by the step's first kernel and
                            read by the rest; one block per stepper (calls on one stream
                            may share it, concurrent steps may not) */
} fgs_step_buffers;

/* Renders view `view` of geom from the n Gaussians in `params` (device SoA,
 * updated in place), takes the L1 term of Eq. 5 against gt[det_h][det_w]
 * (device) plus ssim_weight times its SSIM term, backpropagates through the
 * rasterizer (fgs_project_views_bwd over the forward's lists); with a crop
 * grid and tv_weight > 0, voxelizes the crop, takes tv_weight times its TV
 * and adds the voxelizer backward of that term to the gradient; then one
 * Adam step (fgs_adam_step's arithmetic, densities clamped at 0) on all
 * parameters with moments m, v (device, same layout, updated in place).
 * `grad` (device, same layout) receives the step's gradient. opts: kappa,
 * near plane, model, density_aabb_tau of the rasterizer (the crop's
 * voxelizer takes kappa only); opts->events must be NULL. Workspaces: the
 * rasterizer's (its lists are left there), the crop voxelizer's, and one
 * for the loss terms (with SSIM 12 bytes per pixel, with a crop 44 bytes per
 * Gaussian for the crop's gradient, plus 8 bytes per 16 x 16 detector tile
 * and 8 KiB; ws_loss->needed gives the figure). With
 * key_capacity > 0 in ws_proj and ws_crop the step never waits for the GPU.
 * With a crop, its voxelization, TV and voxelizer backward (into the loss
 * workspace) run on a second stream that the library keeps per device,
 * forked from `stream` after the step's first kernel and joined back before
 * Adam (HIP events), so they overlap with the view's forward and backward;
 * Adam adds the two gradients.
 * The gradient is the one the separate calls give (fgs_l1_loss_grad, then
 * fgs_ssim_loss_grad accumulating, ...) bit for bit; the reported loss
 * terms are the same sums added up in another order (the L1 term per
 * 16 x 16 tile when SSIM is on), so they can differ in the last bits.
 * Same error protocol as the calls it makes: on FGS_E_CAPACITY grow the
 * named workspace and retry; on any error the parameters and moments are
 * unchanged (scratch buffers may have been written). */
int fgs_recon_step(fgs_gaussians_out *params, fgs_gaussian_grads *m, fgs_gaussian_grads *v,
                   fgs_gaussian_grads *grad, int64_t n, const fgs_geom *geom, int32_t view, const float *gt,
                   const fgs_grid *crop, const fgs_opts *opts, const fgs_step_params *sp,
                   const fgs_step_buffers *buf, fgs_workspace *ws_proj, fgs_workspace *ws_crop,
                   fgs_workspace *ws_loss, void *stream);

/* The same step of one view captured in a HIP graph and replayed, for loops
 * that take many steps per view (400 epochs of 75 views in Sec. 4): a step
 * is then two small kernels (the per-call values into buf->params, and
 * Adam) and two graph launches instead of about thirty-five kernel launches.
 *
 * fgs_step_graph_capture takes fgs_recon_step's arguments (all of them
 * fixed for the graph's life: buffers, workspaces and their capacities,
 * view, gt, the loss weights, learning rates and crop dims), records the
 * step without running it (two graphs, the crop branch and the view's
 * forward, loss and backward, and the arguments of the Adam launch), and
 * returns a handle.
 * Requires key_capacity > 0 in ws_proj and, with a crop, in ws_crop (a
 * captured step may not wait for the GPU). Errors as fgs_recon_step (on
 * FGS_E_CAPACITY grow the named workspace and capture again); no graph is
 * returned on error.
 * fgs_step_graph_launch runs one step of the captured view on `stream`:
 * sp->step (Adam's step count) and crop->origin may change from launch to
 * launch, nothing else is read from sp and crop (crop dims must equal the
 * captured ones). The result is the one fgs_recon_step gives with the same
 * values, bit for bit. Asynchronous; launches on one stream run in order.
 * Like fgs_recon_step with a crop, it runs the crop branch on the library's
 * second stream of the device (forked from and joined back into `stream`
 * with events); steps issued from several host threads at once are
 * serialised while they are enqueued.
 * fgs_step_graph_destroy frees the graph (NULL: no-op); it must not be
 * running. Graphs hold the device pointers they were captured with: free or
 * reallocate none of them (or change a workspace's capacity) while a graph
 * that uses them exists. */
typedef struct fgs_step_graph fgs_step_graph;
int fgs_step_graph_capture(fgs_gaussians_out *params, fgs_gaussian_grads *m, fgs_gaussian_grads *v,
                           fgs_gaussian_grads *grad, int64_t n, const fgs_geom *geom, int32_t view,
                           const float *gt, const fgs_grid *crop, const fgs_opts *opts,
                           const fgs_step_params *sp, const fgs_step_buffers *buf, fgs_workspace *ws_proj,
                           fgs_workspace *ws_crop, fgs_workspace *ws_loss, fgs_step_graph **out);
int fgs_step_graph_launch(fgs_step_graph *graph, const fgs_step_params *sp, const fgs_grid *crop, void *stream);
int fgs_step_graph_destroy(fgs_step_graph *graph);

/* ---------------------------------------------------------------------
 * Adaptive density control (Sec. 3.4: the loss gradient prunes, clones or
 * splits Gaussians; Suppl. C: the count is capped 10% above the initial one).
 * ------------------------------------------------------------------- */

/* Per optimiser step: stat[0][i] += |grad_mean_i| (Euclidean norm of
 * grad_mean[3][n]), stat[1][i] += 1 if that norm is > 0 (device, FP32).
 * The caller zeroes stat after each densification. Asynchronous. */
int fgs_adc_accumulate(const float *grad_mean, int64_t n, float *stat, void *stream);

typedef struct {
  float grad_threshold;  /* densify Gaussians whose mean accumulated |dL/dmean| (stat[0] /
                            max(stat[1], 1)) is > this */
  float split_scale;     /* candidates whose largest standard deviation is > this are split,
                            the others cloned (> 0) */
  float prune_density;   /* Gaussians with density < this are removed */
  float prune_scale;     /* and those whose largest standard deviation is > this (> 0) */
  float split_shrink;    /* children's standard deviations = parent's / split_shrink (> 0) */
  int32_t reserved;
  int64_t n_max;         /* cap on the output count */
} fgs_adc_params;

/* One densification step over n = g->n Gaussians with Adam moments m, v
 * (same layout) and statistics stat[2][n] (all device).
 * Each Gaussian is pruned (density < prune_density, or largest standard
 * deviation > prune_scale, or a NaN in either), kept, or, if not pruned and
 * its score exceeds grad_threshold, densified: cloned (two copies at half
 * the density) or, if its largest standard deviation exceeds split_scale,
 * split into two children at mean + R diag(s) z with z from normals[6][n]
 * (device, standard normal variates: rows 0-2 for the first child, 3-5 for
 * the second), log-scales reduced by log(split_shrink), density times
 * split_shrink^3 / 2 (the pair keeps the parent's mass). Clone and split
 * both keep the total mass; every output Gaussian carries its source's
 * Adam moments.
 * If the candidates exceed n_max minus the survivors, those with the largest
 * score are densified (ties: lower index) and the rest kept.
 * Output (device, caller-owned, room for n_max Gaussians): the survivors in
 * input order, each densified one followed by its copy (clone) or with its
 * two children in its place (split), in [3][n_out] / [4][n_out] / [n_out]
 * layout with n_out = *n_out (host) the new count. FGS_E_INVALID if the
 * survivors alone exceed n_max (nothing is written). Waits on the stream once.
 * Workspace: about 25 bytes per Gaussian (FGS_E_CAPACITY protocol). */
int fgs_adc_densify(const fgs_gaussians *g, const fgs_gaussian_grads *m, const fgs_gaussian_grads *v,
                    const float *stat, const float *normals, const fgs_adc_params *p,
                    fgs_gaussians_out *g_out, fgs_gaussian_grads *m_out, fgs_gaussian_grads *v_out,
                    int64_t *n_out, fgs_workspace *ws, void *stream);

/* ---------------------------------------------------------------------
 * Voxelizer (Eq. 2, Sec. 3.3). vol[nz][ny][nx] (device, overwritten) =
 * sum_i rho_i exp(-1/2 d_i^2) [d_i^2 <= kappa^2] at each voxel centre.
 * Gaussians are binned into 8x8x8-voxel tiles with the same scan / sort /
 * range machinery as the rasterizer. Same workspace protocol and single
 * synchronisation as fgs_project_views_fwd.
 * ------------------------------------------------------------------- */
int fgs_voxelize_fwd(const fgs_gaussians *g, const fgs_grid *grid, const fgs_opts *opts, float *vol,
                     fgs_workspace *ws, void *stream);

/* Backward of fgs_voxelize_fwd given grad_vol[nz][ny][nx] (device). */
int fgs_voxelize_bwd(const fgs_gaussians *g, const fgs_grid *grid, const fgs_opts *opts,
                     const float *grad_vol, fgs_gaussian_grads *out, fgs_workspace *ws,
                     void *stream);

/* ---------------------------------------------------------------------
 * Workspace sizing. For op (FGS_OP_*) on n = g->n Gaussians and, for the
 * rasterizer, view_count views of geom with opts (the model matters: the
 * ray-exact model's records and pair slots are twice as large), or, for the
 * voxelizer, grid: a call that bins K (tile, Gaussian) pairs needs at most
 * *fixed_bytes + K * *bytes_per_key bytes of workspace (host outputs). K is
 * known only once the records are built: ws->n_pairs after a call gives it
 * for the same inputs. Only g->n is read from g. Pure host arithmetic; no
 * GPU work, no synchronisation. FGS_E_INVALID on a null pointer, n <= 0,
 * an empty detector or grid, a view count outside [1, geom->n_views] or an
 * unknown op.
 * ------------------------------------------------------------------- */
#define FGS_OP_PROJECT_FWD 0
#define FGS_OP_PROJECT_BWD 1
#define FGS_OP_VOXELIZE_FWD 2
#define FGS_OP_VOXELIZE_BWD 3
int fgs_workspace_query(int32_t op, const fgs_gaussians *g, const fgs_geom *geom, const fgs_grid *grid,
                        int32_t view_count, const fgs_opts *opts, uint64_t *fixed_bytes, uint64_t *bytes_per_key);

/* ---------------------------------------------------------------------
 * Work counters (measurement). The algorithmic work of the rasterizer is
 * the number of (pixel, Gaussian) pairs inside the support (d^2 <= kappa^2,
 * pixels inside the detector); of the voxelizer, the (voxel, Gaussian)
 * pairs. These calls build the same lists as the forward calls and write
 * that count to out[0] (device uint64, overwritten). Same workspace
 * protocol and synchronisation as the forward calls.
 * ------------------------------------------------------------------- */
int fgs_project_views_support(const fgs_gaussians *g, const fgs_geom *geom, int32_t view_begin,
                              int32_t view_count, const fgs_opts *opts, uint64_t *out,
                              fgs_workspace *ws, void *stream);
int fgs_voxelize_support(const fgs_gaussians *g, const fgs_grid *grid, const fgs_opts *opts,
                         uint64_t *out, fgs_workspace *ws, void *stream);

/* ---------------------------------------------------------------------
 * Losses and optimiser (Eq. 5 L1 term; Adam).
 * ------------------------------------------------------------------- */

/* L1 term of Eq. 5 over n_views images of n_per_view values:
 * loss[0] = sum_v mean_pixels |img - gt| (device scalar, overwritten) and
 * grad = sign(img - gt) / n_per_view (device, overwritten; sign(0) = 0).
 * grad may be NULL. Deterministic two-level FP32 reduction (compensated
 * per-thread sums, then pairwise trees); scratch from ws (needs 4 KiB). */
int fgs_l1_loss_grad(const float *img, const float *gt, int64_t n_per_view, int32_t n_views,
                     float *loss, float *grad, fgs_workspace *ws, void *stream);

/* One Adam step (Kingma and Ba, with bias correction, step >= 1) on n
 * float32 values, in place. The gradient is grad + grad2 (grad2 may be
 * NULL): the sum of two loss terms' gradients is fused into the update.
 * m, v are the moment buffers (device). If clamp_min_zero != 0 the updated
 * parameter is clamped at 0 (used for densities). */
int fgs_adam_step(float *param, const float *grad, const float *grad2, float *m, float *v, int64_t n,
                  int32_t step, float lr, float beta1, float beta2, float eps, int32_t clamp_min_zero,
                  void *stream);

/* PSNR = 10 log10(peak^2 / mean((vol - ref)^2)) over n values, written to
 * out[0] (device float). peak > 0 is given by the caller (max of the
 * reference). FP32 reduction as in fgs_l1_loss_grad; scratch from ws
 * (4 KiB). */
int fgs_psnr(const float *vol, const float *ref, int64_t n, float peak, float *out,
             fgs_workspace *ws, void *stream);

/* SSIM term of Eq. 5 over n_views images [n_views][H][W] (device):
 * loss[0] = scale * (1 - mean SSIM(img, gt)) with the local statistics of
 * an 11-tap Gaussian window (sigma 1.5, zero outside the image) and the
 * constants c1, c2 > 0 (0.01^2 and 0.03^2 for unit dynamic range). If grad
 * != NULL it receives scale * d(1 - mean SSIM)/d img, added to its contents
 * when accumulate != 0 (e.g. onto the L1 gradient), else overwriting them.
 * Workspace: 12 bytes per pixel (with grad) plus 4 per 16x16 tile. */
int fgs_ssim_loss_grad(const float *img, const float *gt, int32_t W, int32_t H, int32_t n_views, float c1,
                       float c2, float scale, float *loss, float *grad, int32_t accumulate, fgs_workspace *ws,
                       void *stream);

/* 3D SSIM term of the fitting loss (Eq. 6) over vol, gt [nz][ny][nx]
 * (device): loss[0] = scale * (1 - mean SSIM) with the separable 11^3
 * Gaussian window (sigma 1.5, zero outside the grid), constants c1, c2 > 0;
 * grad (optional) as in fgs_ssim_loss_grad. dims = {nx, ny, nz} (host).
 * Workspace: 40 bytes per voxel. */
int fgs_ssim3d_loss_grad(const float *vol, const float *gt, const int32_t dims[3], float c1, float c2, float scale,
                         float *loss, float *grad, int32_t accumulate, fgs_workspace *ws, void *stream);

/* 3D total variation of vol[nz][ny][nx] (the TV term of Eq. 5, on the
 * sampled sub-volume): loss[0] = scale * (1/n) sum over voxels and axes of
 * |V(i + e_a) - V(i)| (forward differences inside the grid, n = voxel
 * count), and, if grad != NULL, grad = its gradient (sign(0) = 0), both
 * device buffers, overwritten. dims = {nx, ny, nz} (host). Workspace: at
 * most 8 KiB. */
int fgs_tv_loss_grad(const float *vol, const int32_t dims[3], float scale, float *loss, float *grad,
                     fgs_workspace *ws, void *stream);

/* dst[0..n) = src[0..n) (device, FP32, 16-byte aligned, n a multiple of 4):
 * a plain streaming copy that reads and writes exactly 4 n bytes, the
 * reference for scaling HBM traffic counters of the other kernels. */
int fgs_copy(const float *src, float *dst, int64_t n, void *stream);

/* ---------------------------------------------------------------------
 * Measurement probes: the ceilings the pixel and voxel kernels are measured
 * against. fgs_probe launches one register-resident kernel of `blocks`
 * workgroups of 256 threads, each thread running `iters` iterations, and
 * writes one float per thread to sink[blocks * 256] (device; a checksum that
 * keeps the work alive). *work (host) receives the work the launch does, in
 * the unit of its kind:
 *   FGS_PROBE_FMA        FP32 flops of non-packed fused multiply-adds (2 each)
 *   FGS_PROBE_EXP        v_exp_f32 lane operations
 *   FGS_PROBE_FWD_BODY   (pixel, Gaussian) pairs through the splat forward's
 *                        per-pixel arithmetic (exponent by two FMAs down an
 *                        8-pixel column, exp, cutoff select, weighted sum); the
 *                        voxelizer forward's per-voxel body is the same
 *   FGS_PROBE_BWD_BODY   pairs through the splat backward's per-pixel
 *                        arithmetic (two FMAs, exp with cutoff select, three
 *                        accumulating FMAs, per-row and per-pair moment work);
 *                        the voxelizer backward's per-voxel body is the same
 *   FGS_PROBE_LDS        bytes read from LDS by conflict-free ds_read_b128
 *   FGS_PROBE_MFMA_BF16  flops of v_mfma_f32_32x32x16_bf16
 * Time the launch with events on `stream`. Asynchronous. FGS_E_INVALID for
 * an unknown kind or non-positive sizes.
 * ------------------------------------------------------------------- */
#define FGS_PROBE_FMA 0
#define FGS_PROBE_EXP 1
#define FGS_PROBE_FWD_BODY 2
#define FGS_PROBE_BWD_BODY 3
#define FGS_PROBE_LDS 4
#define FGS_PROBE_MFMA_BF16 5
int fgs_probe(int32_t kind, int32_t blocks, int32_t iters, float *sink, double *work, void *stream);

/* ---------------------------------------------------------------------
 * Synthetic ground truth (additive ellipsoid phantom, computed in FP64).
 * ------------------------------------------------------------------- */

/* Exact chord projections: img[view_count][det_h][det_w] = sum_e amp_e *
 * chord length of the ray through each pixel centre. */
int fgs_phantom_project(const fgs_phantom *ph, const fgs_geom *geom, int32_t view_begin,
                        int32_t view_count, float *img, void *stream);

/* Indicator sum at voxel centres: vol[nz][ny][nx]. */
int fgs_phantom_voxelize(const fgs_phantom *ph, const fgs_grid *grid, float *vol, void *stream);

/* ---------------------------------------------------------------------
 * Initialisation (Sec. 3.1).
 * ------------------------------------------------------------------- */

/* FDK reconstruction of a full circular cone-beam scan: projections
 * img[view_count][det_h][det_w] (device) of views [view_begin, view_begin +
 * view_count), which must cover 360 degrees uniformly, into vol[nz][ny][nx]
 * (device, overwritten) on `grid`. Discretisation: cosine pre-weight, a
 * Ram-Lak ramp filter along detector rows by direct convolution on the
 * detector rescaled to the rotation axis, and distance-weighted
 * backprojection with bilinear interpolation and a factor 1/2 for the
 * doubly measured rays. Cone beam only (FGS_E_UNSUPPORTED otherwise);
 * at most 1024 views and 8192 pixels per row. Workspace: view_count *
 * det_h * det_w floats (FGS_E_CAPACITY protocol). No synchronisation. */
int fgs_fdk(const float *img, const fgs_geom *geom, int32_t view_begin, int32_t view_count,
            const fgs_grid *grid, float *vol, fgs_workspace *ws, void *stream);

/* FDK-gradient sampling initialisation of n Gaussians from vol[nz][ny][nx]
 * (device) on `grid` (Sec. 3.1): voxels below background_fraction * max(vol)
 * are zeroed; the gradient magnitude (central differences, zero outside the
 * grid) is quantised to 24 bits of its maximum, and draw i takes the voxel
 * whose cumulative-weight interval holds floor(u0[i] * total weight); the
 * mean is that voxel's corner + (u1, u2, u3)[i] * spacing. uniforms is
 * device double [4][n] of U[0, 1) variates (u0: voxel, u1..u3: position in
 * the voxel). density = density_scale * vol trilinearly interpolated at the
 * mean (zero outside), quaternion = (1, 0, 0, 0), every log-scale = log of
 * the distance to the nearest other mean, floored at min_scale. Writes all
 * four arrays of `out` (device). Waits on the stream once (to check that
 * the volume has a gradient; FGS_E_INVALID if it has none). */
int fgs_gradient_init(const float *vol, const fgs_grid *grid, float background_fraction,
                      float density_scale, float min_scale, int64_t n, const double *uniforms,
                      fgs_gaussians_out *out, fgs_workspace *ws, void *stream);

/* FDK-intensity sampling initialisation, the baseline the paper compares its
 * gradient rule against (Sec. 4, initialisation evaluation): as
 * fgs_gradient_init, with the weight of a voxel its thresholded value itself
 * (voxels below background_fraction * max(vol), and negative ones, weigh
 * zero), quantised to 24 bits of the maximum. FGS_E_INVALID if no voxel has
 * weight. Same arguments, outputs, workspace protocol and single wait. */
int fgs_intensity_init(const float *vol, const fgs_grid *grid, float background_fraction,
                       float density_scale, float min_scale, int64_t n, const double *uniforms,
                       fgs_gaussians_out *out, fgs_workspace *ws, void *stream);

/* ---------------------------------------------------------------------
 * Learned initializer: an MLP (544 -> 128 -> 128 -> 32, 8 outputs used)
 * mapping an FDK patch and position to a Gaussian's density, log-scales and
 * rotation, in BF16 with FP32 accumulation on the matrix cores. BF16 values
 * are stored as uint16_t bit patterns (round to nearest even). Matrices are
 * row-major; "t" buffers hold the transpose (batch index contiguous), which
 * the weight-gradient products read. `rows` is the batch padded to a
 * multiple of 32; padded rows must carry zero features (the gather writes
 * them) and get zero gradient (the heads write it).
 * ------------------------------------------------------------------- */
typedef struct {
  int32_t k_in, hidden, n_out;          /* must be 544, 128, 32 */
  const uint16_t *w1, *w1t;             /* bf16 [128][544] and [544][128] */
  const uint16_t *w2, *w2t;             /* bf16 [128][128] and transpose */
  const uint16_t *w3, *w3t;             /* bf16 [32][128] and [128][32] */
  const float *b1, *b2, *b3;            /* [128], [128], [32] */
} fgs_mlp;

typedef struct {
  float *z1, *z2, *z3;                  /* pre-activations [rows][128], [rows][128], [rows][32] */
  uint16_t *h1, *h1t, *h2, *h2t;        /* bf16 ReLU activations [rows][128] and transposes
                                           (transposes may be NULL when no backward follows) */
} fgs_mlp_acts;

typedef struct {
  float *dw1, *db1, *dw2, *db2, *dw3, *db3;  /* same shapes as the FP32 weights; overwritten */
} fgs_mlp_grads;

/* Features of n Gaussians for the MLP: an 8^3 patch of vol[nz][ny][nx] on
 * `grid`, trilinear samples one voxel apart centred on the mean (zero
 * outside), times inv_norm (divided by norm_max[0] when norm_max, a device
 * scalar such as fgs_reduce_max's output, is not NULL); then 2 * mean
 * (x, y, z); then n_extra (0..29) per-sample values extra[n_extra][n]
 * (device); zeros to 544. Writes x[rows][544] and, if xt != NULL,
 * xt[544][rows] (bf16); rows >= n, a multiple of 32, rows past n are zero.
 * mean is [3][n]. */
int fgs_gather_patches(const float *vol, const fgs_grid *grid, float inv_norm, const float *norm_max,
                       const float *mean, const float *extra, int32_t n_extra, int64_t n, int32_t rows,
                       uint16_t *x, uint16_t *xt, void *stream);

/* bf16 copies w_b[n_out][k_in] and (if w_bt != NULL) w_bt[k_in][n_out] of
 * FP32 weights w[n_out][k_in]. */
int fgs_mlp_pack(const float *w, int32_t n_out, int32_t k_in, uint16_t *w_b, uint16_t *w_bt, void *stream);

/* Forward of the three layers for x[rows][544]: z = x w^T + b, ReLU on the
 * two hidden layers, activations rounded to bf16 between layers. */
int fgs_mlp_fwd(const fgs_mlp *net, const uint16_t *x, int32_t rows, fgs_mlp_acts *acts, void *stream);

/* Prediction heads and loss on z3 (the first n of `rows` rows):
 * density = softplus(z0), log-scales b + z1..z3 with b = base_log_scale[m]
 * (device [n], or 0 when NULL: the network then predicts an offset from a
 * per-sample base such as the nearest-neighbour scale), rotation
 * (z4..z7)/|.|. If params_out != NULL it receives [8][n] (density, 3
 * log-scales, 4 quaternion). If target != NULL ([n][8]: density, log-scales
 * sorted in descending order, unit quaternion with w >= 0) the mean over n
 * of (rho - rho_t)^2 + live * (|s - s_t|^2 + (1 - (q . q_t)^2)), with
 * live = [rho_t > 1e-3] (a fitted Gaussian of no density has no meaningful
 * shape), goes to loss[0] and its gradient with respect to z3 to
 * dz3[rows][32] and dz3t[32][rows] (bf16, zero on padded rows and unused
 * columns). Workspace: ceil(rows/256) floats. */
int fgs_mlp_heads(const float *z3, int32_t rows, int64_t n, const float *base_log_scale, const float *target,
                  float *params_out, uint16_t *dz3, uint16_t *dz3t, float *loss, fgs_workspace *ws,
                  void *stream);

/* Backward of fgs_mlp_fwd: weight and bias gradients (FP32) from the bf16
 * output gradient dz3 (and its transpose), the transposed input xt and the
 * forward's activations. Workspace: 4 * rows * 128 bf16. */
int fgs_mlp_bwd(const fgs_mlp *net, const uint16_t *xt, int32_t rows, const fgs_mlp_acts *acts,
                const uint16_t *dz3, const uint16_t *dz3t, fgs_mlp_grads *grads, fgs_workspace *ws,
                void *stream);

/* Training targets [n][8] (device, overwritten) from fitted Gaussians:
 * density, log-scales in descending order, and the unit quaternion (w >= 0)
 * of the rotation whose columns are permuted to that order (the third
 * negated if needed to keep it proper). (s, R) and (P s, R P^T) describe the
 * same covariance and q, -q the same rotation, so this is the canonical
 * representative the loss compares with. */
int fgs_canonical_targets(const fgs_gaussians *g, float *out, void *stream);

/* out[0] (device) = max of x[0..n) (FP32; the normaliser of the MLP's
 * patch features, Sec. 3.1 init from an FDK volume). Needs 4 KiB of
 * workspace. */
int fgs_reduce_max(const float *x, int64_t n, float *out, fgs_workspace *ws, void *stream);

/* ---------------------------------------------------------------------
 * Introspection (tests): where the last binning of a workspace lives.
 * Pure host arithmetic on the workspace's out fields. After
 * fgs_project_views_fwd / fgs_voxelize_fwd the workspace holds, at the byte
 * offsets written to off[]:
 *   off[0] records' FP32 centres (float2 per record; voxelizer: float4
 *          x, y, z in voxel units and rho),
 *   off[1] FP32 support half-extents (float2 per record, pixels; voxelizer:
 *          float4, voxels),
 *   off[2] tile rectangles (4 x uint16 per record: x0, y0, x1, y1;
 *          voxelizer: 8 x uint16: x0, y0, z0, x1, y1, z1, 0, 0),
 *   off[3] exclusive offsets (uint32, records + 1),
 *   off[4] emitted keys (uint32, pairs), off[5] emitted values (uint32),
 *   off[6] sorted keys, off[7] sorted values, off[8] rasterizer: per tile
 *   (local_view * tiles_per_view + tile) its [begin, end) in the sorted
 *   arrays (2 x uint32, tiles); voxelizer: tile starts (uint32, tiles + 1).
 * counts[0] = records, counts[1] = pairs, counts[2] = tiles.
 * Records are r = local_view * n + i (voxelizer: r = i). Rasterizer keys are
 * local_view << ws->tile_bits | tile, sorted by tile and then view (each
 * key's pairs contiguous, in ascending record order); voxelizer keys are the
 * tile index, sorted ascending. Rasterizer workspaces with ws->record_bits > 0
 * hold one-word lists instead: off[4] and off[5] (off[6] and off[7]) both
 * name the emitted (sorted) words tile << record_bits | r, from which the key
 * is (r / ws->n_gauss) << tile_bits | tile and the value r.
 * ------------------------------------------------------------------- */
int fgs_binning_layout(const fgs_workspace *ws, uint64_t off[9], uint64_t counts[3]);

/* Thread-local message describing the last error (never NULL). */
const char *fgs_last_error(void);

/* Library version string. */
const char *fgs_version(void);

#ifdef __cplusplus
}
#endif

#endif /* FACTGS_H */
