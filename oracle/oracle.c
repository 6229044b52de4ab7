/*
 * FP64 CPU oracle for the Gaussian X-ray rasterizer and voxelizer.
 *
 * TEST INFRASTRUCTURE ONLY. This file is the independent reference that the
 * HIP path is checked against. Only the test suite, the smoke check and the
 * benchmark's CPU-baseline leg may load it; the product path never does.
 * It shares no code, header, table or constant with the HIP library.
 *
 * Everything is plain double-precision C, written for readability rather
 * than speed: per-pixel and per-voxel sums are evaluated directly, OpenMP
 * only splits independent outputs across threads.
 *
 * What it computes (paper sections and equations):
 *   - the Gaussian kernel and its covariance from scale and rotation (Eq. 1);
 *   - the attenuation field as a plain sum of Gaussians (Eq. 2), evaluated at
 *     voxel centres with the 3-sigma (Mahalanobis) support (Sec. 3.3);
 *   - the exact line integral of each Gaussian along a cone-beam or
 *     parallel-beam ray (Eq. 3), and the ray-exact model: that integral with
 *     the kappa support, as an image and with its gradient;
 *   - the method's splat model: each Gaussian projected to a 2D Gaussian on
 *     the detector with the integration factor mu (Eq. 4, Sec. 3.2), summed
 *     in any order (Sec. 3.5, no depth ordering);
 *   - analytic gradients of both with the support held fixed;
 *   - an additive ellipsoid phantom and its exact chord projections, used as
 *     synthetic ground truth.
 *
 * Readings where the paper is silent or garbled:
 *   - support: a pair contributes iff its Mahalanobis distance d^2 <= kappa^2
 *     (kappa = 3); the printed "3 lambda_max" bound is dimensionally a
 *     variance, so the ellipse reading is used;
 *   - ray space: the local affine (EWA-style) map whose third axis is the
 *     Euclidean distance along the ray;
 *   - mu: marginalising the ray-space Gaussian along the ray axis gives
 *     mu = sqrt(2 pi det(S~) / det(S~[0:2,0:2]));
 *   - pixel values are point samples at pixel centres.
 *
 * Geometry (shared description, computed independently here): view k at
 * angle th has its source at SOD (cos th, sin th, 0); camera rows
 * e0 = (-sin th, cos th, 0), e1 = (0, 0, -1), e2 = (-cos th, -sin th, 0);
 * camera coordinates t = W (p - src). A camera point maps to detector pixel
 * coordinates (Fu t0/t2 + det_w/2 + off_u, Fv t1/t2 + det_h/2 + off_v) with
 * Fu = SDD/pitch_u. Pixel (j, i) is sampled at (j + 1/2, i + 1/2).
 * Parallel beam: t = W p and (t0/pitch_u + det_w/2 + off_u, ...).
 *
 * Geometry vector g[] (doubles): 0 mode (0 cone, 1 parallel), 1 sod, 2 sdd,
 * 3 det_w, 4 det_h, 5 pitch_u, 6 pitch_v, 7 off_u, 8 off_v, 9 near.
 * Grid vector gr[] (doubles): origin[3], spacing[3], dims[3] (nx, ny, nz);
 * voxel (i,j,k) centre = origin + (index + 1/2) * spacing; volumes are stored
 * [nz][ny][nx].
 * Gaussians are structure-of-arrays: mean[3][n], log_scale[3][n],
 * quat[4][n] (w, x, y, z; normalised here), density[n].
 */
#include <math.h>
#include <omp.h>
#include <stdlib.h>
#include <string.h>

/* Thread count of the parallel loops (timing at one thread and at all
 * host cores); no arithmetic. */
void orc_set_threads(int n) { omp_set_num_threads(n > 0 ? n : omp_get_num_procs()); }
int orc_max_threads(void) { return omp_get_max_threads(); }

#define TWO_PI 6.283185307179586476925286766559

/* ------------------------------------------------------------------ */
/* small dense linear algebra (row-major 3x3 and 2x2)                 */
/* ------------------------------------------------------------------ */

static void mat3_mul(const double A[9], const double B[9], double C[9]) {
  double T[9];
  for (int i = 0; i < 3; ++i)
    for (int j = 0; j < 3; ++j) {
      double s = 0.0;
      for (int k = 0; k < 3; ++k) s += A[3 * i + k] * B[3 * k + j];
      T[3 * i + j] = s;
    }
  memcpy(C, T, sizeof(T));
}

static void mat3_transpose(const double A[9], double T[9]) {
  double U[9];
  for (int i = 0; i < 3; ++i)
    for (int j = 0; j < 3; ++j) U[3 * j + i] = A[3 * i + j];
  memcpy(T, U, sizeof(U));
}

/* C = A * B * A^T */
static void mat3_sandwich(const double A[9], const double B[9], double C[9]) {
  double AB[9], At[9];
  mat3_mul(A, B, AB);
  mat3_transpose(A, At);
  mat3_mul(AB, At, C);
}

static double mat3_det(const double A[9]) {
  return A[0] * (A[4] * A[8] - A[5] * A[7]) - A[1] * (A[3] * A[8] - A[5] * A[6]) +
         A[2] * (A[3] * A[7] - A[4] * A[6]);
}

/* inverse by the adjugate */
static void mat3_inv(const double A[9], double I[9]) {
  double d = mat3_det(A);
  double J[9];
  J[0] = (A[4] * A[8] - A[5] * A[7]) / d;
  J[1] = (A[2] * A[7] - A[1] * A[8]) / d;
  J[2] = (A[1] * A[5] - A[2] * A[4]) / d;
  J[3] = (A[5] * A[6] - A[3] * A[8]) / d;
  J[4] = (A[0] * A[8] - A[2] * A[6]) / d;
  J[5] = (A[2] * A[3] - A[0] * A[5]) / d;
  J[6] = (A[3] * A[7] - A[4] * A[6]) / d;
  J[7] = (A[1] * A[6] - A[0] * A[7]) / d;
  J[8] = (A[0] * A[4] - A[1] * A[3]) / d;
  memcpy(I, J, sizeof(J));
}

static void mat2_inv(const double A[4], double I[4]) {
  double d = A[0] * A[3] - A[1] * A[2];
  double J[4] = {A[3] / d, -A[1] / d, -A[2] / d, A[0] / d};
  memcpy(I, J, sizeof(J));
}

/* ------------------------------------------------------------------ */
/* Eq. 1: covariance from scale and rotation                           */
/* ------------------------------------------------------------------ */

/* Rotation matrix of the normalised quaternion (w, x, y, z), Hamilton. */
static void quat_rot(const double q_in[4], double R[9], double qn[4], double *qnorm) {
  double n = sqrt(q_in[0] * q_in[0] + q_in[1] * q_in[1] + q_in[2] * q_in[2] + q_in[3] * q_in[3]);
  double w = q_in[0] / n, x = q_in[1] / n, y = q_in[2] / n, z = q_in[3] / n;
  R[0] = 1 - 2 * (y * y + z * z); R[1] = 2 * (x * y - w * z);     R[2] = 2 * (x * z + w * y);
  R[3] = 2 * (x * y + w * z);     R[4] = 1 - 2 * (x * x + z * z); R[5] = 2 * (y * z - w * x);
  R[6] = 2 * (x * z - w * y);     R[7] = 2 * (y * z + w * x);     R[8] = 1 - 2 * (x * x + y * y);
  if (qn) { qn[0] = w; qn[1] = x; qn[2] = y; qn[3] = z; }
  if (qnorm) *qnorm = n;
}

typedef struct {
  double p[3];      /* mean */
  double s2[3];     /* variances along the principal axes */
  double R[9];      /* rotation */
  double qn[4];     /* normalised quaternion */
  double qnorm;     /* |q| of the raw input */
  double Sig[9];    /* covariance R diag(s2) R^T */
  double rho;       /* density */
} gauss3;

static void load_gauss(long n, long i, const double *mean, const double *ls, const double *quat,
                       const double *dens, gauss3 *G) {
  double q[4] = {quat[i], quat[n + i], quat[2 * n + i], quat[3 * n + i]};
  for (int a = 0; a < 3; ++a) {
    G->p[a] = mean[a * n + i];
    G->s2[a] = exp(2.0 * ls[a * n + i]);
  }
  quat_rot(q, G->R, G->qn, &G->qnorm);
  double D[9] = {G->s2[0], 0, 0, 0, G->s2[1], 0, 0, 0, G->s2[2]};
  mat3_sandwich(G->R, D, G->Sig);
  G->rho = dens[i];
}

/* ------------------------------------------------------------------ */
/* View geometry                                                       */
/* ------------------------------------------------------------------ */

typedef struct {
  int parallel;
  double W[9];      /* rows e0, e1, e2 */
  double src[3];    /* source position (cone) */
  double Fu, Fv;    /* cone: SDD / pitch; parallel: 1 / pitch */
  double cu, cv;    /* principal point in pixel coordinates */
  double sdd, pitch_u, pitch_v, near_plane;
} view_t;

static void make_view(const double *g, double th, view_t *V) {
  double c = cos(th), s = sin(th);
  V->parallel = (int)g[0] == 1;
  double W[9] = {-s, c, 0, 0, 0, -1, -c, -s, 0};
  memcpy(V->W, W, sizeof(W));
  V->src[0] = g[1] * c; V->src[1] = g[1] * s; V->src[2] = 0.0;
  V->sdd = g[2];
  V->pitch_u = g[5]; V->pitch_v = g[6];
  V->Fu = V->parallel ? 1.0 / g[5] : g[2] / g[5];
  V->Fv = V->parallel ? 1.0 / g[6] : g[2] / g[6];
  V->cu = 0.5 * g[3] + g[7];
  V->cv = 0.5 * g[4] + g[8];
  V->near_plane = g[9];
}

/* ------------------------------------------------------------------ */
/* Eq. 4: one Gaussian projected to a 2D splat in one view             */
/* ------------------------------------------------------------------ */

typedef struct {
  int culled;
  double t[3];       /* camera coordinates */
  double J[9];       /* ray-space Jacobian at t */
  double M[9];       /* J W */
  double St[9];      /* S~ = M Sigma M^T */
  double St2[4];     /* S~[0:2,0:2] */
  double Sh[4];      /* S^ = D S~2 D */
  double C[4];       /* conic S^^-1 */
  double mu;         /* integration factor */
  double w;          /* rho * mu */
  double uv[2];      /* projected centre in pixel coordinates */
} splat_t;

static void project_gauss(const view_t *V, const gauss3 *G, splat_t *S) {
  double d[3] = {G->p[0] - (V->parallel ? 0.0 : V->src[0]),
                 G->p[1] - (V->parallel ? 0.0 : V->src[1]),
                 G->p[2] - (V->parallel ? 0.0 : V->src[2])};
  for (int a = 0; a < 3; ++a)
    S->t[a] = V->W[3 * a] * d[0] + V->W[3 * a + 1] * d[1] + V->W[3 * a + 2] * d[2];
  S->culled = 0;
  const double *t = S->t;
  if (V->parallel) {
    double I[9] = {1, 0, 0, 0, 1, 0, 0, 0, 1};
    memcpy(S->J, I, sizeof(I));
    S->uv[0] = V->Fu * t[0] + V->cu;
    S->uv[1] = V->Fv * t[1] + V->cv;
  } else {
    if (t[2] <= V->near_plane) { S->culled = 1; return; }
    double L = sqrt(t[0] * t[0] + t[1] * t[1] + t[2] * t[2]);
    double J[9] = {1.0 / t[2], 0.0, -t[0] / (t[2] * t[2]),
                   0.0, 1.0 / t[2], -t[1] / (t[2] * t[2]),
                   t[0] / L, t[1] / L, t[2] / L};
    memcpy(S->J, J, sizeof(J));
    S->uv[0] = V->Fu * t[0] / t[2] + V->cu;
    S->uv[1] = V->Fv * t[1] / t[2] + V->cv;
  }
  mat3_mul(S->J, V->W, S->M);
  mat3_sandwich(S->M, G->Sig, S->St);
  S->St2[0] = S->St[0]; S->St2[1] = S->St[1]; S->St2[2] = S->St[3]; S->St2[3] = S->St[4];
  S->Sh[0] = V->Fu * V->Fu * S->St2[0];
  S->Sh[1] = V->Fu * V->Fv * S->St2[1];
  S->Sh[2] = V->Fv * V->Fu * S->St2[2];
  S->Sh[3] = V->Fv * V->Fv * S->St2[3];
  double dSh = S->Sh[0] * S->Sh[3] - S->Sh[1] * S->Sh[2];
  if (!(dSh > 0.0)) { S->culled = 1; return; }
  mat2_inv(S->Sh, S->C);
  double det3 = mat3_det(S->St);
  double det2 = S->St2[0] * S->St2[3] - S->St2[1] * S->St2[2];
  S->mu = sqrt(TWO_PI * det3 / det2);
  S->w = G->rho * S->mu;
}

static double splat_d2(const splat_t *S, double u, double v) {
  double du = u - S->uv[0], dv = v - S->uv[1];
  return S->C[0] * du * du + (S->C[1] + S->C[2]) * du * dv + S->C[3] * dv * dv;
}

/* Conservative FP64 pixel-coordinate box of the support ellipse. */
static void splat_box(const splat_t *S, double kappa, double box[4]) {
  double ru = kappa * sqrt(S->Sh[0]), rv = kappa * sqrt(S->Sh[3]);
  box[0] = S->uv[0] - ru; box[1] = S->uv[0] + ru;
  box[2] = S->uv[1] - rv; box[3] = S->uv[1] + rv;
}

/* Support of one splat or voxel Gaussian whose contribution peaks at `peak`
 * (w = rho mu for a splat, rho for the voxelizer). Sec. 3.2 keeps pairs with
 * d^2 <= kappa^2; Sec. 3.5 bounds splats by boxes that also take the
 * density into account, read here as also dropping the pairs whose contribution
 * peak exp(-d^2/2) is below tau: d^2 <= min(kappa^2, 2 ln(peak / tau)), whose
 * axis-aligned box shrinks as the peak falls. tau = 0: the kappa support.
 * Returns the bound on d^2, or -1 when the Gaussian contributes nothing
 * (peak <= tau). kappa may be infinite (no cut). */
static double support_k2(double kappa, double tau, double peak) {
  double k2 = kappa * kappa;
  if (tau > 0.0) {
    if (!(peak > tau)) return -1.0;
    const double t = 2.0 * log(peak / tau);
    if (t < k2) k2 = t;
  }
  return k2;
}

/* ------------------------------------------------------------------ */
/* Exported: per-(view, Gaussian) splat records                        */
/* ------------------------------------------------------------------ */

/* Record r = v * n + i. Outputs: uv[2R], Shat[3R] (a, b, c), conic[3R]
 * (C00, C01, C11), mu[R], w[R], culled[R]. */
void orc_splat_records(const double *g, int n_views, const double *angles, long n,
                       const double *mean, const double *ls, const double *quat,
                       const double *dens, double *uv, double *Shat, double *conic,
                       double *mu, double *w, int *culled) {
  for (int v = 0; v < n_views; ++v) {
    view_t V;
    make_view(g, angles[v], &V);
#pragma omp parallel for schedule(static)
    for (long i = 0; i < n; ++i) {
      gauss3 G;
      splat_t S;
      load_gauss(n, i, mean, ls, quat, dens, &G);
      project_gauss(&V, &G, &S);
      long r = (long)v * n + i;
      culled[r] = S.culled;
      if (S.culled) {
        uv[2 * r] = uv[2 * r + 1] = 0; Shat[3 * r] = Shat[3 * r + 1] = Shat[3 * r + 2] = 0;
        conic[3 * r] = conic[3 * r + 1] = conic[3 * r + 2] = 0; mu[r] = w[r] = 0;
        continue;
      }
      uv[2 * r] = S.uv[0]; uv[2 * r + 1] = S.uv[1];
      Shat[3 * r] = S.Sh[0]; Shat[3 * r + 1] = S.Sh[1]; Shat[3 * r + 2] = S.Sh[3];
      conic[3 * r] = S.C[0]; conic[3 * r + 1] = S.C[1]; conic[3 * r + 2] = S.C[3];
      mu[r] = S.mu; w[r] = S.w;
    }
  }
}

/* ------------------------------------------------------------------ */
/* Exported: the method's projection M (Eq. 4 with the kappa support)  */
/* ------------------------------------------------------------------ */

/* Brute force: every pixel of every view sums over every Gaussian.
 * img[n_views][det_h][det_w]. */
void orc_project_brute(const double *g, double kappa, double tau, int n_views, const double *angles, long n,
                       const double *mean, const double *ls, const double *quat,
                       const double *dens, double *img) {
  int W = (int)g[3], H = (int)g[4];
  splat_t *S = (splat_t *)malloc(sizeof(splat_t) * (size_t)n);
  for (int v = 0; v < n_views; ++v) {
    view_t V;
    make_view(g, angles[v], &V);
    for (long i = 0; i < n; ++i) {
      gauss3 G;
      load_gauss(n, i, mean, ls, quat, dens, &G);
      project_gauss(&V, &G, &S[i]);
    }
    double *out = img + (size_t)v * W * H;
#pragma omp parallel for schedule(static)
    for (int y = 0; y < H; ++y)
      for (int x = 0; x < W; ++x) {
        double acc = 0.0;
        for (long i = 0; i < n; ++i) {
          if (S[i].culled) continue;
          const double k2i = support_k2(kappa, tau, S[i].w);
          double d2 = splat_d2(&S[i], x + 0.5, y + 0.5);
          if (k2i >= 0.0 && d2 <= k2i) acc += S[i].w * exp(-0.5 * d2);
        }
        out[(size_t)y * W + x] = acc;
      }
  }
  free(S);
}

/* Gaussian-major variant: each Gaussian visits only the pixels of its FP64
 * support box; the per-pixel test is the same as the brute force, so the
 * result is the same sum (in Gaussian order per pixel). Rows are split
 * across threads; each row sums its Gaussians in ascending index.
 * With band_img != NULL, band_img receives per pixel the sum of the
 * contributions w exp(-d^2/2) of the pairs with |d^2 - kappa^2| <= band
 * (those inside the support are also in img): any evaluation whose support
 * decision errs only on such pairs differs from img by at most band_img. */
static void project_boxed(const double *g, double kappa, double tau, int n_views, const double *angles,
                          long n, const double *mean, const double *ls, const double *quat,
                          const double *dens, double band, double *img, double *band_img) {
  int W = (int)g[3], H = (int)g[4];
  splat_t *S = (splat_t *)malloc(sizeof(splat_t) * (size_t)n);
  double *box = (double *)malloc(sizeof(double) * 4 * (size_t)n);
  double *k2s = (double *)malloc(sizeof(double) * (size_t)n);
  for (int v = 0; v < n_views; ++v) {
    view_t V;
    make_view(g, angles[v], &V);
#pragma omp parallel for schedule(static)
    for (long i = 0; i < n; ++i) {
      gauss3 G;
      load_gauss(n, i, mean, ls, quat, dens, &G);
      project_gauss(&V, &G, &S[i]);
      k2s[i] = S[i].culled ? -1.0 : support_k2(kappa, tau, S[i].w);
      if (k2s[i] >= 0.0) splat_box(&S[i], sqrt(k2s[i] + (band_img ? band : 0.0)), box + 4 * i);
    }
    double *out = img + (size_t)v * W * H;
    double *bout = band_img ? band_img + (size_t)v * W * H : NULL;
#pragma omp parallel for schedule(dynamic, 4)
    for (int y = 0; y < H; ++y) {
      double *row = out + (size_t)y * W;
      double *brow = bout ? bout + (size_t)y * W : NULL;
      for (int x = 0; x < W; ++x) row[x] = 0.0;
      if (brow)
        for (int x = 0; x < W; ++x) brow[x] = 0.0;
      double yc = y + 0.5;
      for (long i = 0; i < n; ++i) {
        const double k2 = k2s[i];
        if (k2 < 0.0) continue;
        const double *b = box + 4 * i;
        if (yc < b[2] || yc > b[3]) continue;
        int x0 = (int)floor(b[0] - 0.5), x1 = (int)ceil(b[1] - 0.5);
        if (x0 < 0) x0 = 0;
        if (x1 > W - 1) x1 = W - 1;
        for (int x = x0; x <= x1; ++x) {
          double d2 = splat_d2(&S[i], x + 0.5, yc);
          if (d2 <= k2) row[x] += S[i].w * exp(-0.5 * d2);
          if (brow && fabs(d2 - k2) <= band) brow[x] += S[i].w * exp(-0.5 * d2);
        }
      }
    }
  }
  free(S);
  free(box);
  free(k2s);
}

void orc_project(const double *g, double kappa, double tau, int n_views, const double *angles, long n,
                 const double *mean, const double *ls, const double *quat,
                 const double *dens, double *img) {
  project_boxed(g, kappa, tau, n_views, angles, n, mean, ls, quat, dens, 0.0, img, NULL);
}

void orc_project_banded(const double *g, double kappa, double tau, int n_views, const double *angles, long n,
                        const double *mean, const double *ls, const double *quat,
                        const double *dens, double band, double *img, double *band_img) {
  project_boxed(g, kappa, tau, n_views, angles, n, mean, ls, quat, dens, band, img, band_img);
}

/* M of one view at arbitrary detector points (u, v), brute force. */
void orc_project_points(const double *g, double kappa, double tau, double angle, long n, const double *mean,
                        const double *ls, const double *quat, const double *dens, long npts,
                        const double *u, const double *v, double *out) {
  view_t V;
  make_view(g, angle, &V);
  splat_t *S = (splat_t *)malloc(sizeof(splat_t) * (size_t)n);
#pragma omp parallel for schedule(static)
  for (long i = 0; i < n; ++i) {
    gauss3 G;
    load_gauss(n, i, mean, ls, quat, dens, &G);
    project_gauss(&V, &G, &S[i]);
  }
#pragma omp parallel for schedule(static)
  for (long k = 0; k < npts; ++k) {
    double acc = 0.0;
    for (long i = 0; i < n; ++i) {
      if (S[i].culled) continue;
      const double k2i = support_k2(kappa, tau, S[i].w);
      double d2 = splat_d2(&S[i], u[k], v[k]);
      if (k2i >= 0.0 && d2 <= k2i) acc += S[i].w * exp(-0.5 * d2);
    }
    out[k] = acc;
  }
  free(S);
}

/* ------------------------------------------------------------------ */
/* Eq. 3: exact line integral along the physical ray                  */
/* ------------------------------------------------------------------ */

/* Ray through detector point (u, v): origin o and unit direction d. */
static void detector_ray(const view_t *V, double u, double v, double o[3], double d[3]) {
  double xu = (u - V->cu) * V->pitch_u, xv = (v - V->cv) * V->pitch_v;
  const double *e0 = V->W, *e1 = V->W + 3, *e2 = V->W + 6;
  if (V->parallel) {
    for (int a = 0; a < 3; ++a) {
      o[a] = xu * e0[a] + xv * e1[a] - 2.0 * e2[a];
      d[a] = e2[a];
    }
  } else {
    double P[3], nrm = 0.0;
    for (int a = 0; a < 3; ++a) {
      P[a] = V->src[a] + V->sdd * e2[a] + xu * e0[a] + xv * e1[a];
      o[a] = V->src[a];
      d[a] = P[a] - V->src[a];
      nrm += d[a] * d[a];
    }
    nrm = sqrt(nrm);
    for (int a = 0; a < 3; ++a) d[a] /= nrm;
  }
}

/* Integral over the whole line of rho exp(-1/2 (x-p)^T A (x-p)),
 * x = o + t d, |d| = 1, completing the square in t. */
static double line_integral(const gauss3 *G, const double A[9], const double o[3],
                            const double d[3]) {
  double c[3] = {o[0] - G->p[0], o[1] - G->p[1], o[2] - G->p[2]};
  double Ad[3], Ac[3];
  for (int a = 0; a < 3; ++a) {
    Ad[a] = A[3 * a] * d[0] + A[3 * a + 1] * d[1] + A[3 * a + 2] * d[2];
    Ac[a] = A[3 * a] * c[0] + A[3 * a + 1] * c[1] + A[3 * a + 2] * c[2];
  }
  double dAd = d[0] * Ad[0] + d[1] * Ad[1] + d[2] * Ad[2];
  double dAc = d[0] * Ac[0] + d[1] * Ac[1] + d[2] * Ac[2];
  double cAc = c[0] * Ac[0] + c[1] * Ac[1] + c[2] * Ac[2];
  return G->rho * sqrt(TWO_PI / dAd) * exp(-0.5 * (cAc - dAc * dAc / dAd));
}

void orc_exact_points(const double *g, double angle, long n, const double *mean, const double *ls,
                      const double *quat, const double *dens, long npts, const double *u,
                      const double *v, double *out) {
  view_t V;
  make_view(g, angle, &V);
#pragma omp parallel for schedule(static)
  for (long k = 0; k < npts; ++k) {
    double o[3], d[3], acc = 0.0;
    detector_ray(&V, u[k], v[k], o, d);
    for (long i = 0; i < n; ++i) {
      gauss3 G;
      double A[9];
      load_gauss(n, i, mean, ls, quat, dens, &G);
      mat3_inv(G.Sig, A);
      acc += line_integral(&G, A, o, d);
    }
    out[k] = acc;
  }
}

/* Origin and unit direction of the ray through detector points, for
 * quadrature drivers: o[3*npts], d[3*npts]. */
void orc_rays(const double *g, double angle, long npts, const double *u, const double *v,
              double *o, double *d) {
  view_t V;
  make_view(g, angle, &V);
  for (long k = 0; k < npts; ++k) detector_ray(&V, u[k], v[k], o + 3 * k, d + 3 * k);
}

/* ------------------------------------------------------------------ */
/* Ray-exact model: Eq. 3 with the kappa support                       */
/* ------------------------------------------------------------------ */

/* The ray-exact model replaces the splat M by the exact line integral E of
 * each Gaussian, with the same kind of support: Gaussian i contributes to
 * the ray through a detector point iff the ray passes within Mahalanobis
 * distance kappa of its mean, i.e. the smallest value over the line of
 * (x - p)^T Sigma^-1 (x - p) is <= kappa^2. In cone beam a Gaussian is left
 * out of a view, as for M, when its camera depth is <= near, and also when
 * the source lies inside its kappa-ellipsoid (then every ray through the
 * source passes within kappa and the support is no longer a bounded region
 * of the detector). */
static void sigma_to_params(const gauss3 *G, const double dSig[9], double dls[3], double dq[4]);

static int exact_valid(const view_t *V, const gauss3 *G, const double A[9], double kappa) {
  if (V->parallel) return 1;
  double x0[3], t2 = 0.0, q = 0.0;
  for (int a = 0; a < 3; ++a) {
    x0[a] = V->src[a] - G->p[a];
    t2 += V->W[6 + a] * (G->p[a] - V->src[a]);
  }
  if (!(t2 > V->near_plane)) return 0;
  for (int a = 0; a < 3; ++a)
    for (int b = 0; b < 3; ++b) q += x0[a] * A[3 * a + b] * x0[b];
  return q > kappa * kappa;
}

/* Quadratic-in-t pieces of (o + t d - p)^T A (o + t d - p), |d| = 1. */
typedef struct {
  double a, b, c, h;   /* d^T A d, d^T A x0, x0^T A x0, c - b^2/a (x0 = o - p) */
  double x0[3], Ad[3], Ax0[3];
} ray_form;

static void ray_form_of(const gauss3 *G, const double A[9], const double o[3], const double d[3],
                        ray_form *F) {
  for (int a = 0; a < 3; ++a) F->x0[a] = o[a] - G->p[a];
  for (int a = 0; a < 3; ++a) {
    F->Ad[a] = A[3 * a] * d[0] + A[3 * a + 1] * d[1] + A[3 * a + 2] * d[2];
    F->Ax0[a] = A[3 * a] * F->x0[0] + A[3 * a + 1] * F->x0[1] + A[3 * a + 2] * F->x0[2];
  }
  F->a = d[0] * F->Ad[0] + d[1] * F->Ad[1] + d[2] * F->Ad[2];
  F->b = d[0] * F->Ax0[0] + d[1] * F->Ax0[1] + d[2] * F->Ax0[2];
  F->c = F->x0[0] * F->Ax0[0] + F->x0[1] * F->Ax0[1] + F->x0[2] * F->Ax0[2];
  F->h = F->c - F->b * F->b / F->a;
}

/* A superset of the detector pixels whose rays meet Gaussian G's
 * kappa-ellipsoid: the image of its bounding ball (radius kappa s_max).
 * Cone beam: a camera point t within r of the centre t_c has
 * |t0/t2 - t0c/t2c| <= r (t2c + |t0c|) / ((t2c - r) t2c), likewise for t1.
 * Returns 0 (use the whole detector) when the ball reaches the source plane. */
static int ball_box(const view_t *V, const gauss3 *G, double kappa, int Wd, int Hd, int box[4]) {
  double smax = sqrt(fmax(G->s2[0], fmax(G->s2[1], G->s2[2])));
  double r = kappa * smax, t[3];
  for (int a = 0; a < 3; ++a) {
    t[a] = 0.0;
    for (int b = 0; b < 3; ++b) t[a] += V->W[3 * a + b] * (G->p[b] - (V->parallel ? 0.0 : V->src[b]));
  }
  double cu, cv, hu, hv;
  if (V->parallel) {
    cu = V->Fu * t[0] + V->cu; cv = V->Fv * t[1] + V->cv;
    hu = V->Fu * r; hv = V->Fv * r;
  } else {
    if (!(t[2] - r > 0.0)) return 0;
    cu = V->Fu * t[0] / t[2] + V->cu; cv = V->Fv * t[1] / t[2] + V->cv;
    hu = V->Fu * r * (t[2] + fabs(t[0])) / ((t[2] - r) * t[2]);
    hv = V->Fv * r * (t[2] + fabs(t[1])) / ((t[2] - r) * t[2]);
  }
  box[0] = (int)floor(cu - hu - 1.5); box[1] = (int)ceil(cu + hu + 0.5);
  box[2] = (int)floor(cv - hv - 1.5); box[3] = (int)ceil(cv + hv + 0.5);
  if (box[0] < 0) box[0] = 0;
  if (box[2] < 0) box[2] = 0;
  if (box[1] > Wd - 1) box[1] = Wd - 1;
  if (box[3] > Hd - 1) box[3] = Hd - 1;
  return 1;
}

/* img[n_views][det_h][det_w] of the ray-exact model. brute != 0: every
 * pixel against every Gaussian; else pixels inside each Gaussian's ball box. */
void orc_exact_project(const double *g, double kappa, int n_views, const double *angles, long n,
                       const double *mean, const double *ls, const double *quat, const double *dens,
                       int brute, double *img) {
  int Wd = (int)g[3], Hd = (int)g[4];
  double k2 = kappa * kappa;
  gauss3 *Gs = (gauss3 *)malloc(sizeof(gauss3) * (size_t)n);
  double *As = (double *)malloc(sizeof(double) * 9 * (size_t)n);
  for (long i = 0; i < n; ++i) {
    load_gauss(n, i, mean, ls, quat, dens, &Gs[i]);
    mat3_inv(Gs[i].Sig, As + 9 * i);
  }
  for (int v = 0; v < n_views; ++v) {
    view_t V;
    make_view(g, angles[v], &V);
    double *out = img + (size_t)v * Wd * Hd;
    if (brute) {
#pragma omp parallel for schedule(static)
      for (long k = 0; k < (long)Wd * Hd; ++k) {
        double o[3], d[3], acc = 0.0;
        detector_ray(&V, (double)(k % Wd) + 0.5, (double)(k / Wd) + 0.5, o, d);
        for (long i = 0; i < n; ++i) {
          if (!exact_valid(&V, &Gs[i], As + 9 * i, kappa)) continue;
          ray_form F;
          ray_form_of(&Gs[i], As + 9 * i, o, d, &F);
          if (F.h <= k2) acc += Gs[i].rho * sqrt(TWO_PI / F.a) * exp(-0.5 * F.h);
        }
        out[k] = acc;
      }
      continue;
    }
    int *bx = (int *)malloc(sizeof(int) * 5 * (size_t)n);
#pragma omp parallel for schedule(static)
    for (long i = 0; i < n; ++i) {
      int *b = bx + 5 * i;
      b[4] = exact_valid(&V, &Gs[i], As + 9 * i, kappa);
      b[0] = 0; b[1] = Wd - 1; b[2] = 0; b[3] = Hd - 1;
      if (b[4]) ball_box(&V, &Gs[i], kappa, Wd, Hd, b);
    }
    /* each thread owns whole rows; Gaussians are visited in index order */
#pragma omp parallel for schedule(dynamic, 1)
    for (int y = 0; y < Hd; ++y) {
      for (int x = 0; x < Wd; ++x) out[(size_t)y * Wd + x] = 0.0;
      for (long i = 0; i < n; ++i) {
        const int *box = bx + 5 * i;
        if (!box[4] || y < box[2] || y > box[3]) continue;
        for (int x = box[0]; x <= box[1]; ++x) {
          double o[3], d[3];
          detector_ray(&V, x + 0.5, y + 0.5, o, d);
          ray_form F;
          ray_form_of(&Gs[i], As + 9 * i, o, d, &F);
          if (F.h <= k2) out[(size_t)y * Wd + x] += Gs[i].rho * sqrt(TWO_PI / F.a) * exp(-0.5 * F.h);
        }
      }
    }
    free(bx);
  }
  free(Gs);
  free(As);
}

/* The ray-exact model at arbitrary detector points of one view. */
void orc_exact_points_cut(const double *g, double kappa, double angle, long n, const double *mean,
                          const double *ls, const double *quat, const double *dens, long npts,
                          const double *u, const double *v, double *out) {
  view_t V;
  make_view(g, angle, &V);
  double k2 = kappa * kappa;
  gauss3 *Gs = (gauss3 *)malloc(sizeof(gauss3) * (size_t)n);
  double *As = (double *)malloc(sizeof(double) * 9 * (size_t)n);
  int *ok = (int *)malloc(sizeof(int) * (size_t)n);
  for (long i = 0; i < n; ++i) {
    load_gauss(n, i, mean, ls, quat, dens, &Gs[i]);
    mat3_inv(Gs[i].Sig, As + 9 * i);
    ok[i] = exact_valid(&V, &Gs[i], As + 9 * i, kappa);
  }
#pragma omp parallel for schedule(static)
  for (long k = 0; k < npts; ++k) {
    double o[3], d[3], acc = 0.0;
    detector_ray(&V, u[k], v[k], o, d);
    for (long i = 0; i < n; ++i) {
      if (!ok[i]) continue;
      ray_form F;
      ray_form_of(&Gs[i], As + 9 * i, o, d, &F);
      if (F.h <= k2) acc += Gs[i].rho * sqrt(TWO_PI / F.a) * exp(-0.5 * F.h);
    }
    out[k] = acc;
  }
  free(Gs);
  free(As);
  free(ok);
}

/* Gradient of one (ray, Gaussian) term E = rho sqrt(2 pi / a) exp(-h / 2),
 * h = c - b^2 / a, times gg, with respect to the mean, A = Sigma^-1 (full
 * 3x3, symmetrised by the caller's conversion) and rho. */
static void exact_term_grad(const gauss3 *G, const ray_form *F, const double d[3], double gg,
                            double dp[3], double dA[9], double *drho) {
  double e1 = sqrt(TWO_PI / F->a) * exp(-0.5 * F->h);
  double E = G->rho * e1;
  *drho += gg * e1;
  double Ea = -0.5 * E * (1.0 / F->a + F->b * F->b / (F->a * F->a));
  double Eb = E * F->b / F->a;
  double Ec = -0.5 * E;
  /* dE/dA = Ea d d^T + Eb d x0^T + Ec x0 x0^T; x0 = o - p, so dE/dp = -dE/dx0 */
  for (int i = 0; i < 3; ++i) {
    for (int j = 0; j < 3; ++j)
      dA[3 * i + j] += gg * (Ea * d[i] * d[j] + Eb * d[i] * F->x0[j] + Ec * F->x0[i] * F->x0[j]);
    dp[i] -= gg * (Eb * F->Ad[i] + 2.0 * Ec * F->Ax0[i]);
  }
}

/* From dL/dA (A = Sigma^-1, full matrix) to the parameter gradients. */
static void exact_chain(const gauss3 *G, const double A[9], const double dA[9], double dls[3], double dq[4]) {
  double sym[9], tmp[9], dSig[9];
  for (int i = 0; i < 3; ++i)
    for (int j = 0; j < 3; ++j) sym[3 * i + j] = 0.5 * (dA[3 * i + j] + dA[3 * j + i]);
  /* A = Sigma^-1: dSigma = -A dA A */
  mat3_mul(A, sym, tmp);
  mat3_mul(tmp, A, dSig);
  for (int e = 0; e < 9; ++e) dSig[e] = -dSig[e];
  sigma_to_params(G, dSig, dls, dq);
}

/* Gradient of sum(grad_img * E_cut) for the Gaussians in sel, the support
 * held fixed; band as in orc_project_bwd, on h - kappa^2. */
void orc_exact_bwd(const double *g, double kappa, int n_views, const double *angles, long n,
                   const double *mean, const double *ls, const double *quat, const double *dens,
                   const double *grad_img, long n_sel, const long *sel, double *dmean, double *dls,
                   double *dq, double *drho, double band, double *band_abs) {
  int Wd = (int)g[3], Hd = (int)g[4];
  double k2 = kappa * kappa;
  view_t *Vs = (view_t *)malloc(sizeof(view_t) * (size_t)n_views);
  for (int v = 0; v < n_views; ++v) make_view(g, angles[v], &Vs[v]);
#pragma omp parallel for schedule(dynamic, 4)
  for (long k = 0; k < n_sel; ++k) {
    gauss3 G;
    double A[9];
    load_gauss(n, sel[k], mean, ls, quat, dens, &G);
    mat3_inv(G.Sig, A);
    double dp[3] = {0, 0, 0}, dA[9] = {0}, r1 = 0.0, babs[11] = {0};
    for (int v = 0; v < n_views; ++v) {
      const view_t *V = &Vs[v];
      if (!exact_valid(V, &G, A, kappa)) continue;
      int box[4] = {0, Wd - 1, 0, Hd - 1};
      ball_box(V, &G, sqrt(k2 + band), Wd, Hd, box);
      const double *gi = grad_img + (size_t)v * Wd * Hd;
      for (int y = box[2]; y <= box[3]; ++y)
        for (int x = box[0]; x <= box[1]; ++x) {
          double o[3], d[3];
          detector_ray(V, x + 0.5, y + 0.5, o, d);
          ray_form F;
          ray_form_of(&G, A, o, d, &F);
          if (F.h > k2 + band) continue;
          double gg = gi[(size_t)y * Wd + x];
          if (band > 0.0 && fabs(F.h - k2) <= band) {
            double p1[3] = {0, 0, 0}, a1[9] = {0}, q1 = 0.0, l3[3], q4[4];
            exact_term_grad(&G, &F, d, gg, p1, a1, &q1);
            exact_chain(&G, A, a1, l3, q4);
            for (int a = 0; a < 3; ++a) { babs[a] += fabs(p1[a]); babs[3 + a] += fabs(l3[a]); }
            for (int c = 0; c < 4; ++c) babs[6 + c] += fabs(q4[c]);
            babs[10] += fabs(q1);
            continue;
          }
          if (F.h > k2) continue;
          exact_term_grad(&G, &F, d, gg, dp, dA, &r1);
        }
    }
    double l3[3], q4[4];
    exact_chain(&G, A, dA, l3, q4);
    for (int a = 0; a < 3; ++a) { dmean[a * n_sel + k] = dp[a]; dls[a * n_sel + k] = l3[a]; }
    for (int c = 0; c < 4; ++c) dq[c * n_sel + k] = q4[c];
    drho[k] = r1;
    if (band_abs)
      for (int c = 0; c < 11; ++c) band_abs[c * n_sel + k] = babs[c];
  }
  free(Vs);
}

/* ------------------------------------------------------------------ */
/* Eq. 2, Sec. 3.3: the density field and the voxelizer                */
/* ------------------------------------------------------------------ */

/* sigma(x) at arbitrary points with the kappa support (kappa <= 0 or
 * infinite means no cutoff): x[3*npts]. */
void orc_field_points(double kappa, double tau, long n, const double *mean, const double *ls,
                      const double *quat, const double *dens, long npts, const double *x,
                      double *out) {
  gauss3 *G = (gauss3 *)malloc(sizeof(gauss3) * (size_t)n);
  double *A = (double *)malloc(sizeof(double) * 9 * (size_t)n);
  for (long i = 0; i < n; ++i) {
    load_gauss(n, i, mean, ls, quat, dens, &G[i]);
    mat3_inv(G[i].Sig, A + 9 * i);
  }
  const double kcut = (kappa > 0 && isfinite(kappa)) ? kappa : INFINITY;
#pragma omp parallel for schedule(static)
  for (long k = 0; k < npts; ++k) {
    double acc = 0.0;
    for (long i = 0; i < n; ++i) {
      double dd[3] = {x[3 * k] - G[i].p[0], x[3 * k + 1] - G[i].p[1], x[3 * k + 2] - G[i].p[2]};
      const double *Ai = A + 9 * i;
      double d2 = 0.0;
      for (int a = 0; a < 3; ++a)
        for (int b = 0; b < 3; ++b) d2 += dd[a] * Ai[3 * a + b] * dd[b];
      const double k2i = support_k2(kcut, tau, G[i].rho);
      if (k2i >= 0.0 && d2 <= k2i) acc += G[i].rho * exp(-0.5 * d2);
    }
    out[k] = acc;
  }
  free(G);
  free(A);
}

static void voxel_centre(const double *gr, long ix, long iy, long iz, double x[3]) {
  x[0] = gr[0] + (ix + 0.5) * gr[3];
  x[1] = gr[1] + (iy + 0.5) * gr[4];
  x[2] = gr[2] + (iz + 0.5) * gr[5];
}

/* Brute force voxelizer: vol[nz][ny][nx]. */
void orc_voxelize_brute(double kappa, double tau, const double *gr, long n, const double *mean,
                        const double *ls, const double *quat, const double *dens, double *vol) {
  long nx = (long)gr[6], ny = (long)gr[7], nz = (long)gr[8];
  long nv = nx * ny * nz;
  double *pts = (double *)malloc(sizeof(double) * 3 * (size_t)nv);
  for (long iz = 0; iz < nz; ++iz)
    for (long iy = 0; iy < ny; ++iy)
      for (long ix = 0; ix < nx; ++ix) voxel_centre(gr, ix, iy, iz, pts + 3 * ((iz * ny + iy) * nx + ix));
  orc_field_points(kappa, tau, n, mean, ls, quat, dens, nv, pts, vol);
  free(pts);
}

/* Box of the support ellipsoid in voxel indices (conservative by one voxel). */
static void vox_box(const double *gr, const gauss3 *G, double kappa, long lo[3], long hi[3]) {
  for (int a = 0; a < 3; ++a) {
    double r = kappa * sqrt(G->Sig[4 * a]);
    double f0 = (G->p[a] - r - gr[a]) / gr[3 + a] - 0.5;
    double f1 = (G->p[a] + r - gr[a]) / gr[3 + a] - 0.5;
    long n = (long)gr[6 + a];
    double l = floor(f0), h = ceil(f1);
    lo[a] = l < 0 ? 0 : (l > n ? n : (long)l);
    hi[a] = h > n - 1 ? n - 1 : (h < -1 ? -1 : (long)h);
  }
}

/* Box-limited voxelizer: each z-slice sums its Gaussians in ascending index.
 * band_vol (optional) as band_img of project_boxed. */
static void voxelize_boxed(double kappa, double tau, const double *gr, long n, const double *mean,
                           const double *ls, const double *quat, const double *dens, double band, double *vol,
                           double *band_vol) {
  long nx = (long)gr[6], ny = (long)gr[7], nz = (long)gr[8];
  gauss3 *G = (gauss3 *)malloc(sizeof(gauss3) * (size_t)n);
  double *A = (double *)malloc(sizeof(double) * 9 * (size_t)n);
  long *bx = (long *)malloc(sizeof(long) * 6 * (size_t)n);
  double *k2s = (double *)malloc(sizeof(double) * (size_t)n);
#pragma omp parallel for schedule(static)
  for (long i = 0; i < n; ++i) {
    load_gauss(n, i, mean, ls, quat, dens, &G[i]);
    mat3_inv(G[i].Sig, A + 9 * i);
    k2s[i] = support_k2(kappa, tau, G[i].rho);
    if (k2s[i] >= 0.0) {
      vox_box(gr, &G[i], sqrt(k2s[i] + (band_vol ? band : 0.0)), bx + 6 * i, bx + 6 * i + 3);
    } else {
      bx[6 * i + 2] = 1; bx[6 * i + 5] = 0;   /* empty z range */
    }
  }
#pragma omp parallel for schedule(dynamic, 1)
  for (long iz = 0; iz < nz; ++iz) {
    double *slab = vol + (size_t)iz * nx * ny;
    double *bslab = band_vol ? band_vol + (size_t)iz * nx * ny : NULL;
    for (long k = 0; k < nx * ny; ++k) slab[k] = 0.0;
    if (bslab)
      for (long k = 0; k < nx * ny; ++k) bslab[k] = 0.0;
    for (long i = 0; i < n; ++i) {
      const long *lo = bx + 6 * i, *hi = bx + 6 * i + 3;
      if (iz < lo[2] || iz > hi[2]) continue;
      const double *Ai = A + 9 * i;
      const double k2 = k2s[i];
      for (long iy = lo[1]; iy <= hi[1]; ++iy)
        for (long ix = lo[0]; ix <= hi[0]; ++ix) {
          double x[3];
          voxel_centre(gr, ix, iy, iz, x);
          double dd[3] = {x[0] - G[i].p[0], x[1] - G[i].p[1], x[2] - G[i].p[2]};
          double d2 = 0.0;
          for (int a = 0; a < 3; ++a)
            for (int b = 0; b < 3; ++b) d2 += dd[a] * Ai[3 * a + b] * dd[b];
          if (d2 <= k2) slab[iy * nx + ix] += G[i].rho * exp(-0.5 * d2);
          if (bslab && fabs(d2 - k2) <= band) bslab[iy * nx + ix] += G[i].rho * exp(-0.5 * d2);
        }
    }
  }
  free(G);
  free(A);
  free(bx);
  free(k2s);
}

void orc_voxelize(double kappa, double tau, const double *gr, long n, const double *mean, const double *ls,
                  const double *quat, const double *dens, double *vol) {
  voxelize_boxed(kappa, tau, gr, n, mean, ls, quat, dens, 0.0, vol, NULL);
}

void orc_voxelize_banded(double kappa, double tau, const double *gr, long n, const double *mean,
                         const double *ls, const double *quat, const double *dens, double band, double *vol,
                         double *band_vol) {
  voxelize_boxed(kappa, tau, gr, n, mean, ls, quat, dens, band, vol, band_vol);
}

/* ------------------------------------------------------------------ */
/* Gradients with the support held fixed                               */
/* ------------------------------------------------------------------ */

/* From dL/dSigma (symmetric 3x3) to dL/d log_scale and dL/d quat. */
static void sigma_to_params(const gauss3 *G, const double dSig[9], double dls[3], double dq[4]) {
  /* Sigma = R diag(s2) R^T: dR = 2 dSig R diag(s2); dls_j = 2 s2_j r_j^T dSig r_j */
  double dR[9];
  for (int i = 0; i < 3; ++i)
    for (int j = 0; j < 3; ++j) {
      double acc = 0.0;
      for (int k = 0; k < 3; ++k) acc += dSig[3 * i + k] * G->R[3 * k + j];
      dR[3 * i + j] = 2.0 * acc * G->s2[j];
    }
  for (int j = 0; j < 3; ++j) {
    double acc = 0.0;
    for (int a = 0; a < 3; ++a)
      for (int b = 0; b < 3; ++b) acc += G->R[3 * a + j] * dSig[3 * a + b] * G->R[3 * b + j];
    dls[j] = 2.0 * G->s2[j] * acc;
  }
  /* R(q) of the normalised quaternion; partial derivatives of each entry. */
  double w = G->qn[0], x = G->qn[1], y = G->qn[2], z = G->qn[3];
  double dRdq[9][4] = {
      {0, 0, -4 * y, -4 * z},         {-2 * z, 2 * y, 2 * x, -2 * w}, {2 * y, 2 * z, 2 * w, 2 * x},
      {2 * z, 2 * y, 2 * x, 2 * w},   {0, -4 * x, 0, -4 * z},         {-2 * x, -2 * w, 2 * z, 2 * y},
      {-2 * y, 2 * z, -2 * w, 2 * x}, {2 * x, 2 * w, 2 * z, 2 * y},   {0, -4 * x, -4 * y, 0}};
  double dqn[4] = {0, 0, 0, 0};
  for (int e = 0; e < 9; ++e)
    for (int c = 0; c < 4; ++c) dqn[c] += dR[e] * dRdq[e][c];
  /* q_hat = q / |q| */
  double dot = dqn[0] * w + dqn[1] * x + dqn[2] * y + dqn[3] * z;
  for (int c = 0; c < 4; ++c) dq[c] = (dqn[c] - G->qn[c] * dot) / G->qnorm;
}

/* Chain rule for one (view, Gaussian) splat, given the sums over its
 * support pixels: sw = sum g e, sp = dL/d uv, sC = dL/dC (full 2x2). Adds
 * into dmean[3], dls[3], dq[4], drho. */
static void splat_backward(const view_t *V, const gauss3 *G, const splat_t *S, double sw,
                           const double sp[2], const double sC[4], double dmean[3], double dls[3],
                           double dq[4], double *drho) {
  *drho += S->mu * sw;
  double dmu = G->rho * sw;
  /* C = Sh^-1 -> dSh = -C dC C */
  double T[4], dSh[4];
  T[0] = sC[0] * S->C[0] + sC[1] * S->C[2]; T[1] = sC[0] * S->C[1] + sC[1] * S->C[3];
  T[2] = sC[2] * S->C[0] + sC[3] * S->C[2]; T[3] = sC[2] * S->C[1] + sC[3] * S->C[3];
  dSh[0] = -(S->C[0] * T[0] + S->C[1] * T[2]); dSh[1] = -(S->C[0] * T[1] + S->C[1] * T[3]);
  dSh[2] = -(S->C[2] * T[0] + S->C[3] * T[2]); dSh[3] = -(S->C[2] * T[1] + S->C[3] * T[3]);
  /* Sh = D S~2 D and mu = sqrt(2 pi det S~ / det S~2) */
  double dSt[9] = {0};
  double Sti[9], St2i[4];
  mat3_inv(S->St, Sti);
  mat2_inv(S->St2, St2i);
  for (int a = 0; a < 9; ++a) dSt[a] = 0.5 * S->mu * dmu * Sti[a];
  dSt[0] += V->Fu * V->Fu * dSh[0] - 0.5 * S->mu * dmu * St2i[0];
  dSt[1] += V->Fu * V->Fv * dSh[1] - 0.5 * S->mu * dmu * St2i[1];
  dSt[3] += V->Fv * V->Fu * dSh[2] - 0.5 * S->mu * dmu * St2i[2];
  dSt[4] += V->Fv * V->Fv * dSh[3] - 0.5 * S->mu * dmu * St2i[3];
  /* S~ = M Sigma M^T: dSigma = M^T dS~ M, dM = 2 dS~ M Sigma */
  double Mt[9], tmp[9], dSig[9], dM[9];
  mat3_transpose(S->M, Mt);
  mat3_mul(Mt, dSt, tmp);
  mat3_mul(tmp, S->M, dSig);
  mat3_mul(dSt, S->M, tmp);
  mat3_mul(tmp, G->Sig, dM);
  for (int a = 0; a < 9; ++a) dM[a] *= 2.0;
  /* camera coordinates t */
  const double *t = S->t;
  double dt[3] = {0, 0, 0};
  if (V->parallel) {
    dt[0] += V->Fu * sp[0];
    dt[1] += V->Fv * sp[1];
  } else {
    /* uv = (Fu t0/t2, Fv t1/t2) + c */
    dt[0] += V->Fu * sp[0] / t[2];
    dt[1] += V->Fv * sp[1] / t[2];
    dt[2] += -(V->Fu * sp[0] * t[0] + V->Fv * sp[1] * t[1]) / (t[2] * t[2]);
    /* M = J W: dJ = dM W^T */
    double Wt[9], dJ[9];
    mat3_transpose(V->W, Wt);
    mat3_mul(dM, Wt, dJ);
    double t2 = t[2], t22 = t2 * t2, t23 = t22 * t2;
    double L = sqrt(t[0] * t[0] + t[1] * t[1] + t[2] * t[2]), L3 = L * L * L;
    /* first two rows */
    dt[2] += -dJ[0] / t22 - dJ[4] / t22;
    dt[0] += -dJ[2] / t22;
    dt[2] += 2.0 * t[0] * dJ[2] / t23;
    dt[1] += -dJ[5] / t22;
    dt[2] += 2.0 * t[1] * dJ[5] / t23;
    /* third row t / L */
    for (int k = 0; k < 3; ++k)
      for (int m = 0; m < 3; ++m)
        dt[m] += dJ[6 + k] * ((k == m ? 1.0 / L : 0.0) - t[k] * t[m] / L3);
  }
  /* t = W (p - src) */
  for (int a = 0; a < 3; ++a)
    dmean[a] += V->W[a] * dt[0] + V->W[3 + a] * dt[1] + V->W[6 + a] * dt[2];
  double l3[3], q4[4];
  sigma_to_params(G, dSig, l3, q4);
  for (int a = 0; a < 3; ++a) dls[a] += l3[a];
  for (int c = 0; c < 4; ++c) dq[c] += q4[c];
}

/* Gradient of L = sum_pixels grad_img * M with respect to the parameters of
 * the Gaussians listed in sel[n_sel] (every Gaussian's gradient depends on
 * its own support only). Outputs are [3][n_sel], [3][n_sel], [4][n_sel],
 * [n_sel]. grad_img is [n_views][det_h][det_w]. */
/* Pairs whose d^2 lies within `band` of kappa^2 sit on the support boundary,
 * where the hard cutoff makes the gradient discontinuous and an evaluation in
 * any finite precision may include or exclude them. With band > 0 they are
 * left out of the gradient and the sum over them of |per-pair gradient| is
 * written to band_abs[11][n_sel] (mean 3, log_scale 3, quat 4, density 1):
 * any implementation's gradient lies within band_abs of the returned one,
 * up to its own rounding. band = 0 gives the plain gradient. */
static void pair_grad_abs(const view_t *V, const gauss3 *G, const splat_t *S, double gg, double du,
                          double dv, double d2, double *acc11) {
  double e = exp(-0.5 * d2);
  double sw = gg * e;
  double cdu = S->C[0] * du + S->C[1] * dv, cdv = S->C[2] * du + S->C[3] * dv;
  double sp[2] = {gg * S->w * e * cdu, gg * S->w * e * cdv};
  double sC[4] = {-0.5 * gg * S->w * e * du * du, -0.5 * gg * S->w * e * du * dv,
                  -0.5 * gg * S->w * e * dv * du, -0.5 * gg * S->w * e * dv * dv};
  double m3[3] = {0, 0, 0}, l3[3] = {0, 0, 0}, q4[4] = {0, 0, 0, 0}, r1 = 0.0;
  splat_backward(V, G, S, sw, sp, sC, m3, l3, q4, &r1);
  for (int a = 0; a < 3; ++a) { acc11[a] += fabs(m3[a]); acc11[3 + a] += fabs(l3[a]); }
  for (int c = 0; c < 4; ++c) acc11[6 + c] += fabs(q4[c]);
  acc11[10] += fabs(r1);
}

void orc_project_bwd(const double *g, double kappa, double tau, int n_views, const double *angles, long n,
                     const double *mean, const double *ls, const double *quat,
                     const double *dens, const double *grad_img, long n_sel, const long *sel,
                     double *dmean, double *dls, double *dq, double *drho, double band,
                     double *band_abs) {
  int W = (int)g[3], H = (int)g[4];
  view_t *Vs = (view_t *)malloc(sizeof(view_t) * (size_t)n_views);
  for (int v = 0; v < n_views; ++v) make_view(g, angles[v], &Vs[v]);
#pragma omp parallel for schedule(dynamic, 16)
  for (long k = 0; k < n_sel; ++k) {
    long i = sel[k];
    gauss3 G;
    load_gauss(n, i, mean, ls, quat, dens, &G);
    double m3[3] = {0, 0, 0}, l3[3] = {0, 0, 0}, q4[4] = {0, 0, 0, 0}, r1 = 0.0;
    double babs[11] = {0};
    for (int v = 0; v < n_views; ++v) {
      splat_t S;
      project_gauss(&Vs[v], &G, &S);
      if (S.culled) continue;
      const double k2 = support_k2(kappa, tau, S.w);
      if (k2 < 0.0) continue;
      double box[4];
      splat_box(&S, sqrt(k2 + band), box);
      int x0 = (int)floor(box[0] - 0.5), x1 = (int)ceil(box[1] - 0.5);
      int y0 = (int)floor(box[2] - 0.5), y1 = (int)ceil(box[3] - 0.5);
      if (x0 < 0) x0 = 0;
      if (y0 < 0) y0 = 0;
      if (x1 > W - 1) x1 = W - 1;
      if (y1 > H - 1) y1 = H - 1;
      const double *gi = grad_img + (size_t)v * W * H;
      double sw = 0.0, sp[2] = {0, 0}, sC[4] = {0, 0, 0, 0};
      for (int y = y0; y <= y1; ++y)
        for (int x = x0; x <= x1; ++x) {
          double du = x + 0.5 - S.uv[0], dv = y + 0.5 - S.uv[1];
          double d2 = splat_d2(&S, x + 0.5, y + 0.5);
          if (d2 > k2 + band) continue;
          double gg = gi[(size_t)y * W + x];
          if (band > 0.0 && fabs(d2 - k2) <= band) {
            pair_grad_abs(&Vs[v], &G, &S, gg, du, dv, d2, babs);
            continue;
          }
          double e = exp(-0.5 * d2);
          sw += gg * e;
          /* d(d2)/d(uv) = -2 C (x - uv): d e / d uv = e C (x - uv) */
          double cdu = S.C[0] * du + S.C[1] * dv, cdv = S.C[2] * du + S.C[3] * dv;
          sp[0] += gg * S.w * e * cdu;
          sp[1] += gg * S.w * e * cdv;
          sC[0] += -0.5 * gg * S.w * e * du * du;
          sC[1] += -0.5 * gg * S.w * e * du * dv;
          sC[2] += -0.5 * gg * S.w * e * dv * du;
          sC[3] += -0.5 * gg * S.w * e * dv * dv;
        }
      splat_backward(&Vs[v], &G, &S, sw, sp, sC, m3, l3, q4, &r1);
    }
    for (int a = 0; a < 3; ++a) { dmean[a * n_sel + k] = m3[a]; dls[a * n_sel + k] = l3[a]; }
    for (int c = 0; c < 4; ++c) dq[c * n_sel + k] = q4[c];
    drho[k] = r1;
    if (band_abs)
      for (int c = 0; c < 11; ++c) band_abs[c * n_sel + k] = babs[c];
  }
  free(Vs);
}

/* Gradient of L = sum_voxels grad_vol * V for the Gaussians in sel. */
/* Same band convention as orc_project_bwd. */
static void voxel_chain(const gauss3 *G, const double A[9], double sr, const double sp[3],
                        const double sA[9], double m3[3], double l3[3], double q4[4], double *r1) {
  /* A = Sigma^-1: dSigma = -A dA A */
  double tmp[9], dSig[9];
  mat3_mul(A, sA, tmp);
  mat3_mul(tmp, A, dSig);
  for (int a = 0; a < 9; ++a) dSig[a] = -dSig[a];
  sigma_to_params(G, dSig, l3, q4);
  for (int a = 0; a < 3; ++a) m3[a] = sp[a];
  *r1 = sr;
}

void orc_voxelize_bwd(double kappa, double tau, const double *gr, long n, const double *mean, const double *ls,
                      const double *quat, const double *dens, const double *grad_vol, long n_sel,
                      const long *sel, double *dmean, double *dls, double *dq, double *drho,
                      double band, double *band_abs) {
  long nx = (long)gr[6], ny = (long)gr[7];
#pragma omp parallel for schedule(dynamic, 16)
  for (long k = 0; k < n_sel; ++k) {
    long i = sel[k];
    gauss3 G;
    double A[9];
    long lo[3], hi[3];
    load_gauss(n, i, mean, ls, quat, dens, &G);
    mat3_inv(G.Sig, A);
    const double k2 = support_k2(kappa, tau, G.rho);
    if (k2 < 0.0) {
      for (int a = 0; a < 3; ++a) { dmean[a * n_sel + k] = 0.0; dls[a * n_sel + k] = 0.0; }
      for (int c = 0; c < 4; ++c) dq[c * n_sel + k] = 0.0;
      drho[k] = 0.0;
      if (band_abs)
        for (int c = 0; c < 11; ++c) band_abs[c * n_sel + k] = 0.0;
      continue;
    }
    vox_box(gr, &G, sqrt(k2 + band), lo, hi);
    double sr = 0.0, sp[3] = {0, 0, 0}, sA[9] = {0};
    double babs[11] = {0};
    for (long iz = lo[2]; iz <= hi[2]; ++iz)
      for (long iy = lo[1]; iy <= hi[1]; ++iy)
        for (long ix = lo[0]; ix <= hi[0]; ++ix) {
          double x[3];
          voxel_centre(gr, ix, iy, iz, x);
          double dd[3] = {x[0] - G.p[0], x[1] - G.p[1], x[2] - G.p[2]};
          double Ad[3];
          for (int a = 0; a < 3; ++a) Ad[a] = A[3 * a] * dd[0] + A[3 * a + 1] * dd[1] + A[3 * a + 2] * dd[2];
          double d2 = dd[0] * Ad[0] + dd[1] * Ad[1] + dd[2] * Ad[2];
          if (d2 > k2 + band) continue;
          double gg = grad_vol[(iz * ny + iy) * nx + ix];
          double e = exp(-0.5 * d2);
          if (band > 0.0 && fabs(d2 - k2) <= band) {
            double psp[3], psA[9], m3[3], l3[3], q4[4], r1;
            for (int a = 0; a < 3; ++a) psp[a] = gg * G.rho * e * Ad[a];
            for (int a = 0; a < 3; ++a)
              for (int b = 0; b < 3; ++b) psA[3 * a + b] = -0.5 * gg * G.rho * e * dd[a] * dd[b];
            voxel_chain(&G, A, gg * e, psp, psA, m3, l3, q4, &r1);
            for (int a = 0; a < 3; ++a) { babs[a] += fabs(m3[a]); babs[3 + a] += fabs(l3[a]); }
            for (int c = 0; c < 4; ++c) babs[6 + c] += fabs(q4[c]);
            babs[10] += fabs(r1);
            continue;
          }
          sr += gg * e;
          for (int a = 0; a < 3; ++a) sp[a] += gg * G.rho * e * Ad[a];
          for (int a = 0; a < 3; ++a)
            for (int b = 0; b < 3; ++b) sA[3 * a + b] += -0.5 * gg * G.rho * e * dd[a] * dd[b];
        }
    double m3[3], l3[3], q4[4], r1;
    voxel_chain(&G, A, sr, sp, sA, m3, l3, q4, &r1);
    for (int a = 0; a < 3; ++a) { dmean[a * n_sel + k] = m3[a]; dls[a * n_sel + k] = l3[a]; }
    for (int c = 0; c < 4; ++c) dq[c * n_sel + k] = q4[c];
    drho[k] = r1;
    if (band_abs)
      for (int c = 0; c < 11; ++c) band_abs[c * n_sel + k] = babs[c];
  }
}

/* ------------------------------------------------------------------ */
/* Ellipsoid phantom (synthetic ground truth)                          */
/* ------------------------------------------------------------------ */

/* Q_e = R diag(1/a^2) R^T for ellipsoid e. */
static void ellipsoid_form(const double *semi, const double *quat, long e, double Q[9]) {
  double R[9];
  double q[4] = {quat[4 * e], quat[4 * e + 1], quat[4 * e + 2], quat[4 * e + 3]};
  quat_rot(q, R, NULL, NULL);
  double D[9] = {1.0 / (semi[3 * e] * semi[3 * e]), 0, 0, 0, 1.0 / (semi[3 * e + 1] * semi[3 * e + 1]), 0,
                 0, 0, 1.0 / (semi[3 * e + 2] * semi[3 * e + 2])};
  mat3_sandwich(R, D, Q);
}

/* Indicator sum at voxel centres; centre[3E], semi[3E], quat[4E], amp[E]. */
void orc_phantom_volume(long n_ell, const double *centre, const double *semi, const double *quat,
                        const double *amp, const double *gr, double *vol) {
  long nx = (long)gr[6], ny = (long)gr[7], nz = (long)gr[8];
  double *Q = (double *)malloc(sizeof(double) * 9 * (size_t)n_ell);
  for (long e = 0; e < n_ell; ++e) ellipsoid_form(semi, quat, e, Q + 9 * e);
#pragma omp parallel for schedule(static)
  for (long iz = 0; iz < nz; ++iz)
    for (long iy = 0; iy < ny; ++iy)
      for (long ix = 0; ix < nx; ++ix) {
        double x[3], acc = 0.0;
        voxel_centre(gr, ix, iy, iz, x);
        for (long e = 0; e < n_ell; ++e) {
          double d[3] = {x[0] - centre[3 * e], x[1] - centre[3 * e + 1], x[2] - centre[3 * e + 2]};
          double f = 0.0;
          for (int a = 0; a < 3; ++a)
            for (int b = 0; b < 3; ++b) f += d[a] * Q[9 * e + 3 * a + b] * d[b];
          if (f <= 1.0) acc += amp[e];
        }
        vol[(iz * ny + iy) * nx + ix] = acc;
      }
  free(Q);
}

/* Exact projection: sum of amplitude times chord length along each ray
 * through a pixel centre. The chord solves (o + t d - c)^T Q (o + t d - c) = 1:
 * A t^2 + 2 B t + C = 0 with A = d^T Q d, B = d^T Q (o - c),
 * C = (o - c)^T Q (o - c) - 1; its length is 2 sqrt(B^2 - A C) / A. */
void orc_phantom_project(const double *g, int n_views, const double *angles, long n_ell,
                         const double *centre, const double *semi, const double *quat,
                         const double *amp, double *img) {
  int W = (int)g[3], H = (int)g[4];
  double *Q = (double *)malloc(sizeof(double) * 9 * (size_t)n_ell);
  for (long e = 0; e < n_ell; ++e) ellipsoid_form(semi, quat, e, Q + 9 * e);
  for (int v = 0; v < n_views; ++v) {
    view_t V;
    make_view(g, angles[v], &V);
#pragma omp parallel for schedule(static)
    for (int y = 0; y < H; ++y)
      for (int x = 0; x < W; ++x) {
        double o[3], d[3], acc = 0.0;
        detector_ray(&V, x + 0.5, y + 0.5, o, d);
        for (long e = 0; e < n_ell; ++e) {
          const double *Qe = Q + 9 * e;
          double oc[3] = {o[0] - centre[3 * e], o[1] - centre[3 * e + 1], o[2] - centre[3 * e + 2]};
          double Qd[3], Qo[3];
          for (int a = 0; a < 3; ++a) {
            Qd[a] = Qe[3 * a] * d[0] + Qe[3 * a + 1] * d[1] + Qe[3 * a + 2] * d[2];
            Qo[a] = Qe[3 * a] * oc[0] + Qe[3 * a + 1] * oc[1] + Qe[3 * a + 2] * oc[2];
          }
          double A = d[0] * Qd[0] + d[1] * Qd[1] + d[2] * Qd[2];
          double B = d[0] * Qo[0] + d[1] * Qo[1] + d[2] * Qo[2];
          double C = oc[0] * Qo[0] + oc[1] * Qo[1] + oc[2] * Qo[2] - 1.0;
          double disc = B * B - A * C;
          if (disc > 0.0) acc += amp[e] * 2.0 * sqrt(disc) / A;
        }
        img[((size_t)v * H + y) * W + x] = acc;
      }
  }
  free(Q);
}
