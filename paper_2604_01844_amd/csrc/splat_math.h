// Per-(view, Gaussian) projection math of the X-ray rasterizer (Eq. 4,
// Sec. 3.2) and its chain rule, FP32, shared by the record kernel and the
// record-gradient kernel.
//
// Forward, for Gaussian (p, s, R, rho) and view frame (rows e0, e1, e2,
// source src):
//   t = W (p - src)                      camera coordinates (cone beam)
//   T = D J2 W                           2x3: detector pixels per unit of
//                                        world displacement at p, where J2 is
//                                        the first two rows of the ray-space
//                                        Jacobian [[1/t2, 0, -t0/t2^2],
//                                        [0, 1/t2, -t1/t2^2]] and
//                                        D = diag(fu, fv) = diag(sdd/pitch)
//   U = T R diag(s), S^ = U U^T          projected covariance (pixels^2)
//   C = S^^-1                            conic
//   mu = sqrt(2 pi / (d^T Sigma^-1 d))   with d the unit ray direction
//                                        through p; this is the ray-axis
//                                        marginal of the ray-space Gaussian,
//                                        computed without forming Sigma^-1:
//                                        d^T Sigma^-1 d = sum_j (r_j . d)^2 / s_j^2
//   w = rho mu, centre (fu t0/t2 + cu, fv t1/t2 + cv).
// Parallel beam: T = diag(1/pitch) [e0; e1], d = e2, centre (t0/pu + cu, ...).
#pragma once

#include "fgs_internal.h"

namespace fgs {

struct GeomDev {
  int mode;
  int det_w, det_h;
  int tiles_x, tiles_y;
  int view_begin;
  float sod;
  float fu, fv;        // cone: sdd / pitch; parallel: 1 / pitch
  float cu, cv;        // principal point (pixels)
  float near_plane;
  float kappa;
  float tau;           // density-aware support threshold (0 = off)
  int ablate;          // FGS_ABLATE_* bits (measurement only)
  const float *angles;
};

struct ViewFrame {
  float e0[3], e1[3], e2[3];
  float src[3];
};

__device__ __forceinline__ void make_frame(const GeomDev &G, int view, ViewFrame &F) {
  float s, c;
  sincosf(G.angles[view], &s, &c);
  F.e0[0] = -s; F.e0[1] = c;   F.e0[2] = 0.f;
  F.e1[0] = 0.f; F.e1[1] = 0.f; F.e1[2] = -1.f;
  F.e2[0] = -c; F.e2[1] = -s;  F.e2[2] = 0.f;
  F.src[0] = G.sod * c; F.src[1] = G.sod * s; F.src[2] = 0.f;
}

struct Splat {
  bool ok;
  float t[3];
  float T[2][3];
  float V[3][3];   // R diag(s)
  float U[2][3];
  float a, b, c;   // S^ = [[a, b], [b, c]]
  float C00, C01, C11;
  float dh[3];     // unit ray direction through the mean
  float L;         // |p - src| (cone), 1 (parallel)
  float aj[3];     // r_j . d
  float Q;
  float mu, w;
  float u, v;
};

__device__ __forceinline__ float dot3(const float a[3], const float b[3]) {
  return a[0] * b[0] + a[1] * b[1] + a[2] * b[2];
}

__device__ __forceinline__ void splat_forward(const GaussParams &P, const ViewFrame &F,
                                              const GeomDev &G, Splat &S) {
  float d[3];
  const bool cone = (G.mode == FGS_CONE);
  for (int a = 0; a < 3; ++a) d[a] = cone ? P.p[a] - F.src[a] : P.p[a];
  S.t[0] = dot3(F.e0, d);
  S.t[1] = dot3(F.e1, d);
  S.t[2] = dot3(F.e2, d);
  S.ok = true;
  if (cone) {
    if (!(S.t[2] > G.near_plane)) {
      S.ok = false;
      return;
    }
    const float it = 1.f / S.t[2];
    const float it2 = it * it;
    for (int a = 0; a < 3; ++a) {
      S.T[0][a] = G.fu * (F.e0[a] * it - S.t[0] * it2 * F.e2[a]);
      S.T[1][a] = G.fv * (F.e1[a] * it - S.t[1] * it2 * F.e2[a]);
    }
    S.u = G.fu * S.t[0] * it + G.cu;
    S.v = G.fv * S.t[1] * it + G.cv;
    S.L = sqrtf(dot3(d, d));
    const float il = 1.f / S.L;
    for (int a = 0; a < 3; ++a) S.dh[a] = d[a] * il;
  } else {
    for (int a = 0; a < 3; ++a) {
      S.T[0][a] = G.fu * F.e0[a];
      S.T[1][a] = G.fv * F.e1[a];
      S.dh[a] = F.e2[a];
    }
    S.u = G.fu * S.t[0] + G.cu;
    S.v = G.fv * S.t[1] + G.cv;
    S.L = 1.f;
  }
  for (int a = 0; a < 3; ++a)
    for (int j = 0; j < 3; ++j) S.V[a][j] = P.R[3 * a + j] * P.s[j];
  for (int k = 0; k < 2; ++k)
    for (int j = 0; j < 3; ++j)
      S.U[k][j] = S.T[k][0] * S.V[0][j] + S.T[k][1] * S.V[1][j] + S.T[k][2] * S.V[2][j];
  S.a = S.U[0][0] * S.U[0][0] + S.U[0][1] * S.U[0][1] + S.U[0][2] * S.U[0][2];
  S.b = S.U[0][0] * S.U[1][0] + S.U[0][1] * S.U[1][1] + S.U[0][2] * S.U[1][2];
  S.c = S.U[1][0] * S.U[1][0] + S.U[1][1] * S.U[1][1] + S.U[1][2] * S.U[1][2];
  const float det = S.a * S.c - S.b * S.b;
  if (!(det > 0.f) || !isfinite(det)) {
    S.ok = false;
    return;
  }
  const float id = 1.f / det;
  S.C00 = S.c * id;
  S.C01 = -S.b * id;
  S.C11 = S.a * id;
  float Q = 0.f;
  for (int j = 0; j < 3; ++j) {
    S.aj[j] = P.R[j] * S.dh[0] + P.R[3 + j] * S.dh[1] + P.R[6 + j] * S.dh[2];
    const float r = S.aj[j] / P.s[j];
    Q += r * r;
  }
  S.Q = Q;
  S.mu = sqrtf(kTwoPi / Q);
  S.w = P.rho * S.mu;
}

// Chain rule from the per-record pixel sums to the 11 parameters.
// sums: s0 = sum g e, s1 = sum g e dx, s2 = sum g e dy, s3 = sum g e dx^2,
// s4 = sum g e dx dy, s5 = sum g e dy^2, with (dx, dy) = pixel - centre and
// e = exp(-d^2/2) over the support. out: dmean[3], dlog_scale[3], dquat[4],
// ddensity.
__device__ __forceinline__ void splat_backward(const GaussParams &P, const ViewFrame &F,
                                               const GeomDev &G, const Splat &S,
                                               const float sums[6], float out[11]) {
  const bool cone = (G.mode == FGS_CONE);
  const float dw = sums[0];
  // centre: d e / d centre = e C (x - centre)
  const float du = S.w * (S.C00 * sums[1] + S.C01 * sums[2]);
  const float dv = S.w * (S.C01 * sums[1] + S.C11 * sums[2]);
  // conic, as a symmetric matrix with independent entries
  const float g00 = -0.5f * S.w * sums[3];
  const float g01 = -0.5f * S.w * sums[4];
  const float g11 = -0.5f * S.w * sums[5];
  // S^ = C^-1: dS^ = -C dC C
  const float m00 = S.C00 * g00 + S.C01 * g01, m01 = S.C00 * g01 + S.C01 * g11;
  const float m10 = S.C01 * g00 + S.C11 * g01, m11 = S.C01 * g01 + S.C11 * g11;
  const float h00 = -(m00 * S.C00 + m01 * S.C01);
  const float h01 = -(m00 * S.C01 + m01 * S.C11);
  const float h11 = -(m10 * S.C01 + m11 * S.C11);
  // S^ = U U^T: dU = 2 dS^ U
  float dU[2][3];
  for (int j = 0; j < 3; ++j) {
    dU[0][j] = 2.f * (h00 * S.U[0][j] + h01 * S.U[1][j]);
    dU[1][j] = 2.f * (h01 * S.U[0][j] + h11 * S.U[1][j]);
  }
  // U = T V: dT = dU V^T, dV = T^T dU
  float dT[2][3], dV[3][3];
  for (int k = 0; k < 2; ++k)
    for (int a = 0; a < 3; ++a) dT[k][a] = dU[k][0] * S.V[a][0] + dU[k][1] * S.V[a][1] + dU[k][2] * S.V[a][2];
  for (int a = 0; a < 3; ++a)
    for (int j = 0; j < 3; ++j) dV[a][j] = S.T[0][a] * dU[0][j] + S.T[1][a] * dU[1][j];
  // V = R diag(s)
  float dR[9], dls[3];
  for (int j = 0; j < 3; ++j) {
    float acc = 0.f;
    for (int a = 0; a < 3; ++a) {
      dR[3 * a + j] = dV[a][j] * P.s[j];
      acc += P.R[3 * a + j] * dV[a][j];
    }
    dls[j] = P.s[j] * acc;
  }
  // w = rho mu, mu = sqrt(2 pi / Q), Q = sum_j (a_j / s_j)^2, a_j = r_j . d
  const float drho = S.mu * dw;
  const float dmu = P.rho * dw;
  const float dQ = dmu * (-0.5f * S.mu / S.Q);
  float gdh[3] = {0.f, 0.f, 0.f};
  for (int j = 0; j < 3; ++j) {
    const float is2 = 1.f / (P.s[j] * P.s[j]);
    const float ga = dQ * 2.f * S.aj[j] * is2;
    dls[j] += dQ * (-2.f * S.aj[j] * S.aj[j] * is2);
    for (int a = 0; a < 3; ++a) {
      dR[3 * a + j] += ga * S.dh[a];
      gdh[a] += ga * P.R[3 * a + j];
    }
  }
  float dmean[3] = {0.f, 0.f, 0.f};
  float dt[3] = {0.f, 0.f, 0.f};
  if (cone) {
    // d = (p - src) / L
    const float proj = dot3(S.dh, gdh);
    for (int a = 0; a < 3; ++a) dmean[a] += (gdh[a] - S.dh[a] * proj) / S.L;
    const float it = 1.f / S.t[2];
    const float it2 = it * it, it3 = it2 * it;
    const float T0e2 = dot3(dT[0], F.e2), T1e2 = dot3(dT[1], F.e2);
    const float T0e0 = dot3(dT[0], F.e0), T1e1 = dot3(dT[1], F.e1);
    dt[0] += -G.fu * it2 * T0e2;
    dt[1] += -G.fv * it2 * T1e2;
    dt[2] += G.fu * (-T0e0 * it2 + 2.f * S.t[0] * it3 * T0e2) +
             G.fv * (-T1e1 * it2 + 2.f * S.t[1] * it3 * T1e2);
    dt[0] += G.fu * du * it;
    dt[1] += G.fv * dv * it;
    dt[2] += -(G.fu * du * S.t[0] + G.fv * dv * S.t[1]) * it2;
  } else {
    dt[0] = G.fu * du;
    dt[1] = G.fv * dv;
  }
  for (int a = 0; a < 3; ++a) dmean[a] += F.e0[a] * dt[0] + F.e1[a] * dt[1] + F.e2[a] * dt[2];
  float dq[4];
  rot_grad_to_quat(P.qh, P.qnorm, dR, dq);
  out[0] = dmean[0]; out[1] = dmean[1]; out[2] = dmean[2];
  out[3] = dls[0]; out[4] = dls[1]; out[5] = dls[2];
  out[6] = dq[0]; out[7] = dq[1]; out[8] = dq[2]; out[9] = dq[3];
  out[10] = drho;
}

}  // namespace fgs
