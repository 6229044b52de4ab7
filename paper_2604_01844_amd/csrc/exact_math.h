// Per-(view, Gaussian) quantities of the ray-exact model (the line integral
// E of Eq. 3 with the kappa support) in cone beam, FP32, and their chain
// rule. Shared by the ray-exact record kernel and record-gradient kernel.
//
// Camera frame: the source at the origin, axes e0, e1 (detector u, v) and e2
// (central ray); t = W (p - src) is the mean in it and A = W Sigma^-1 W^T.
// The ray through detector pixel coordinate (x, y) has direction
// d = (s, r, 1), s = (x - cu) / fu, r = (y - cv) / fv. With the mean's
// projection (u, v) = (fu t0/t2 + cu, fv t1/t2 + cv), d_m = (t0/t2, t1/t2, 1)
// and the pixel offset delta = (x - u, y - v):
//   d = d_m + (delta_x / fu, delta_y / fv, 0)
//   d^T A d = a0 + 2 l.delta + delta^T K delta                   =: A(delta)
//   min over the line of (x - p)^T Sigma^-1 (x - p) = t2^2 C(delta) / A(delta)
//   C = a0 K - l l^T (the Schur form, >= 0)
//   E = rho |d| sqrt(2 pi / A(delta)) exp(-t2^2 C(delta) / (2 A(delta)))
// with, in pixel units, K = D A[0:2,0:2] D, l = D (A d_m)[0:2],
// a0 = d_m^T A d_m, D = diag(1/fu, 1/fv). The minimum follows from putting
// the ray's point at depth t2 at t2 d: its offset from the mean is
// t2 (delta_x / fu, delta_y / fv, 0), and completing the square along d.
// |d| depends on the pixel alone; the pixel kernels apply it.
//
// The support {t2^2 C(delta) <= kappa^2 A(delta)} is the detector image of
// the kappa-ellipsoid: the ellipse (delta - dc)^T M (delta - dc) <= gamma,
// M = t2^2 C - kappa^2 K, dc = kappa^2 M^-1 l, gamma = kappa^2 (a0 + l.dc),
// when the source lies outside the ellipsoid (t2^2 a0 > kappa^2); such
// Gaussians are the only ones the model keeps in a view.
#pragma once

#include "splat_math.h"

namespace fgs {

struct ExactSplat {
  bool ok;
  float t[3];
  float V[3][3];     // V[a][j] = (e_a . r_j) / s_j, so A = V V^T
  float A[3][3];
  float dm[2];       // (t0/t2, t1/t2)
  float Ad[3];       // A d_m
  float a0;
  float K00, K01, K11, lu, lv;
  float C00, C01, C11;
  float u, v;
  float esn;         // -t2^2 / 2
  float w;           // rho sqrt(2 pi)
};

__device__ __forceinline__ void exact_forward(const GaussParams &P, const ViewFrame &F, const GeomDev &G,
                                              ExactSplat &X) {
  float d[3];
  for (int a = 0; a < 3; ++a) d[a] = P.p[a] - F.src[a];
  X.t[0] = dot3(F.e0, d);
  X.t[1] = dot3(F.e1, d);
  X.t[2] = dot3(F.e2, d);
  X.ok = X.t[2] > G.near_plane;
  if (!X.ok) return;
  const float *e[3] = {F.e0, F.e1, F.e2};
  for (int a = 0; a < 3; ++a)
    for (int j = 0; j < 3; ++j)
      X.V[a][j] = (e[a][0] * P.R[j] + e[a][1] * P.R[3 + j] + e[a][2] * P.R[6 + j]) / P.s[j];
  for (int a = 0; a < 3; ++a)
    for (int b = 0; b < 3; ++b) X.A[a][b] = X.V[a][0] * X.V[b][0] + X.V[a][1] * X.V[b][1] + X.V[a][2] * X.V[b][2];
  const float it = 1.f / X.t[2];
  X.dm[0] = X.t[0] * it;
  X.dm[1] = X.t[1] * it;
  for (int a = 0; a < 3; ++a) X.Ad[a] = X.A[a][0] * X.dm[0] + X.A[a][1] * X.dm[1] + X.A[a][2];
  X.a0 = X.dm[0] * X.Ad[0] + X.dm[1] * X.Ad[1] + X.Ad[2];
  const float ifu = 1.f / G.fu, ifv = 1.f / G.fv;
  X.K00 = X.A[0][0] * ifu * ifu;
  X.K01 = X.A[0][1] * ifu * ifv;
  X.K11 = X.A[1][1] * ifv * ifv;
  X.lu = X.Ad[0] * ifu;
  X.lv = X.Ad[1] * ifv;
  X.C00 = X.a0 * X.K00 - X.lu * X.lu;
  X.C01 = X.a0 * X.K01 - X.lu * X.lv;
  X.C11 = X.a0 * X.K11 - X.lv * X.lv;
  X.u = G.fu * X.dm[0] + G.cu;
  X.v = G.fv * X.dm[1] + G.cv;
  X.esn = -0.5f * X.t[2] * X.t[2];
  X.w = P.rho * sqrtf(kTwoPi);
  // the source must lie outside the kappa-ellipsoid: (src - p)^T Sigma^-1 (src - p) = t2^2 a0
  X.ok = (X.t[2] * X.t[2] * X.a0 > G.kappa * G.kappa) && isfinite(X.a0) && X.a0 > 0.f;
}

// The support ellipse on the detector (pixel coordinates) from the record
// coefficients: centre, half-extents of its box, and the conic cs with
// (x - centre)^T cs (x - centre) <= kappa^2 inside. False if degenerate.
__device__ __forceinline__ bool exact_silhouette(float K00, float K01, float K11, float lu, float lv, float a0,
                                                 float C00, float C01, float C11, float t2sq, float k2,
                                                 float &dcx, float &dcy, float &hx, float &hy, float &cs00,
                                                 float &cs01, float &cs11) {
  const float M00 = t2sq * C00 - k2 * K00;
  const float M01 = t2sq * C01 - k2 * K01;
  const float M11 = t2sq * C11 - k2 * K11;
  const float det = M00 * M11 - M01 * M01;
  if (!(M00 > 0.f) || !(det > 0.f) || !isfinite(det)) return false;
  const float id = 1.f / det;
  const float i00 = M11 * id, i01 = -M01 * id, i11 = M00 * id;
  dcx = k2 * (i00 * lu + i01 * lv);
  dcy = k2 * (i01 * lu + i11 * lv);
  const float gam = k2 * (a0 + lu * dcx + lv * dcy);
  if (!(gam > 0.f)) return false;
  hx = sqrtf(gam * i00);
  hy = sqrtf(gam * i11);
  const float sc = k2 / gam;
  cs00 = sc * M00;
  cs01 = sc * M01;
  cs11 = sc * M11;
  return true;
}

// Chain rule from the per-record pixel sums to the 11 parameters. With
// p = g |d| A^-1/2 exp(phi), phi = esn C / A, over the support pixels:
//   s[0] = sum p            s[1] = sum p C / A
//   s[2..7]  = sum alpha {1, dx, dy, dx^2, dx dy, dy^2}, alpha = -(p / A)(1/2 + phi)
//   s[8..12] = sum beta {dx, dy, dx^2, dx dy, dy^2},    beta = p / A
// (dx, dy) = pixel - (u, v). alpha and beta are dE/dA and dE/dC per unit w;
// out: dmean[3], dlog_scale[3], dquat[4], ddensity.
__device__ __forceinline__ void exact_backward(const GaussParams &P, const ViewFrame &F, const GeomDev &G,
                                               const ExactSplat &X, const float s[13], float out[11]) {
  const float W = X.w, esn = X.esn;
  const float al0 = s[2], al1 = s[3], al2 = s[4], al3 = s[5], al4 = s[6], al5 = s[7];
  const float be1 = s[8], be2 = s[9], be3 = s[10], be4 = s[11], be5 = s[12];
  const float gw = s[0];
  const float gesn = W * s[1];
  float ga0 = W * al0;
  float glu = 2.f * W * al1, glv = 2.f * W * al2;
  float gK00 = W * al3, gK01 = 2.f * W * al4, gK11 = W * al5;
  const float gC00 = W * esn * be3, gC01 = 2.f * W * esn * be4, gC11 = W * esn * be5;
  const float gu = -W * (2.f * X.lu * al0 + 2.f * X.K00 * al1 + 2.f * X.K01 * al2 +
                         esn * (2.f * X.C00 * be1 + 2.f * X.C01 * be2));
  const float gv = -W * (2.f * X.lv * al0 + 2.f * X.K01 * al1 + 2.f * X.K11 * al2 +
                         esn * (2.f * X.C01 * be1 + 2.f * X.C11 * be2));
  // C = a0 K - l l^T
  ga0 += gC00 * X.K00 + gC01 * X.K01 + gC11 * X.K11;
  gK00 += X.a0 * gC00;
  gK01 += X.a0 * gC01;
  gK11 += X.a0 * gC11;
  glu += -2.f * X.lu * gC00 - X.lv * gC01;
  glv += -X.lu * gC01 - 2.f * X.lv * gC11;
  // to the camera-frame A (full-matrix gradient) and d_m
  const float ifu = 1.f / G.fu, ifv = 1.f / G.fv;
  const float dv3[3] = {X.dm[0], X.dm[1], 1.f};
  float GA[3][3];
  for (int a = 0; a < 3; ++a)
    for (int b = 0; b < 3; ++b) GA[a][b] = ga0 * dv3[a] * dv3[b];
  for (int b = 0; b < 3; ++b) {
    GA[0][b] += glu * ifu * dv3[b];
    GA[1][b] += glv * ifv * dv3[b];
  }
  GA[0][0] += gK00 * ifu * ifu;
  GA[0][1] += 0.5f * gK01 * ifu * ifv;
  GA[1][0] += 0.5f * gK01 * ifu * ifv;
  GA[1][1] += gK11 * ifv * ifv;
  float gd[2];
  for (int b = 0; b < 2; ++b)
    gd[b] = glu * ifu * X.A[0][b] + glv * ifv * X.A[1][b] + 2.f * ga0 * X.Ad[b];
  // d_m = (t0/t2, t1/t2), (u, v) = (fu, fv) d_m + c, esn = -t2^2/2
  const float gs = gd[0] + G.fu * gu, gr = gd[1] + G.fv * gv;
  const float it = 1.f / X.t[2];
  float dt[3];
  dt[0] = gs * it;
  dt[1] = gr * it;
  dt[2] = -(gs * X.dm[0] + gr * X.dm[1]) * it - X.t[2] * gesn;
  float dmean[3];
  for (int a = 0; a < 3; ++a) dmean[a] = F.e0[a] * dt[0] + F.e1[a] * dt[1] + F.e2[a] * dt[2];
  // A = V V^T with the symmetric part of GA: dV = 2 GS V
  float gV[3][3];
  for (int a = 0; a < 3; ++a)
    for (int j = 0; j < 3; ++j) {
      float acc = 0.f;
      for (int b = 0; b < 3; ++b) acc += (GA[a][b] + GA[b][a]) * X.V[b][j];
      gV[a][j] = acc;
    }
  // V[a][j] = (e_a . r_j) / s_j
  const float *e[3] = {F.e0, F.e1, F.e2};
  float dR[9], dls[3];
  for (int j = 0; j < 3; ++j) {
    float acc = 0.f;
    for (int a = 0; a < 3; ++a) acc += gV[a][j] * X.V[a][j];
    dls[j] = -acc;
    for (int b = 0; b < 3; ++b)
      dR[3 * b + j] = (gV[0][j] * e[0][b] + gV[1][j] * e[1][b] + gV[2][j] * e[2][b]) / P.s[j];
  }
  float dq[4];
  rot_grad_to_quat(P.qh, P.qnorm, dR, dq);
  out[0] = dmean[0]; out[1] = dmean[1]; out[2] = dmean[2];
  out[3] = dls[0]; out[4] = dls[1]; out[5] = dls[2];
  out[6] = dq[0]; out[7] = dq[1]; out[8] = dq[2]; out[9] = dq[3];
  out[10] = sqrtf(kTwoPi) * gw;
}

}  // namespace fgs
