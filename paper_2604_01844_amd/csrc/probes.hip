// Measurement probes: register-resident kernels that give the ceilings the
// roofline of the pixel and voxel kernels is taken against.
//
//   FMA        independent chains of FP32 fused multiply-adds (non-packed:
//              the library is built without two-wide packed FP32);
//   EXP        independent chains of v_exp_f32;
//   FWD_BODY   the splat forward's per-pair arithmetic exactly as its pixel
//              loop does it: per pair the offset and the two expansion
//              coefficients, then per pixel of the lane's 8-pixel column two
//              FMAs for the exponent, one v_exp_f32, the cutoff select and
//              the weighted accumulate. The voxelizer forward's row loop is
//              the same per-voxel body;
//   BWD_BODY   the splat backward's per-pair arithmetic: per row the
//              exponent's row coefficients, per pixel two FMAs, one
//              v_exp_f32 with the cutoff select and three accumulating FMAs
//              (column sum, row sum, cc-weighted row sum), per row three
//              moment FMAs, per pair the column sums and the six moments.
//              The voxelizer backward's body is the same per voxel;
//   LDS        conflict-free ds_read_b128 from LDS, consecutive lanes on
//              consecutive 16-byte words;
//   MFMA_BF16  back-to-back v_mfma_f32_32x32x16_bf16 on four independent
//              accumulators.
//
// The pair constants of the body probes change every iteration (so nothing
// is loop-invariant) and every result feeds a sum written to `sink`, so the
// compiler can drop none of the work.
#include "fgs_internal.h"

namespace fgs {
namespace {

constexpr int kProbeThreads = 256;
typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef float f32x16 __attribute__((ext_vector_type(16)));

__device__ __forceinline__ void write_sink(float *sink, float v) {
  sink[uint64_t(blockIdx.x) * kProbeThreads + threadIdx.x] = v;
}

__global__ __launch_bounds__(kProbeThreads) void probe_fma_kernel(int iters, float a, float b, float *sink) {
  float x[8];
#pragma unroll
  for (int k = 0; k < 8; ++k) x[k] = float(threadIdx.x + k) * 1e-3f;
  for (int it = 0; it < iters; ++it) {
#pragma unroll
    for (int r = 0; r < 4; ++r)
#pragma unroll
      for (int k = 0; k < 8; ++k) x[k] = fmaf(x[k], a, b);
  }
  float s = 0.f;
#pragma unroll
  for (int k = 0; k < 8; ++k) s += x[k];
  write_sink(sink, s);
}

__global__ __launch_bounds__(kProbeThreads) void probe_exp_kernel(int iters, float *sink) {
  float x[8];
#pragma unroll
  for (int k = 0; k < 8; ++k) x[k] = float(threadIdx.x + k) * 1e-3f;
  for (int it = 0; it < iters; ++it) {
#pragma unroll
    for (int r = 0; r < 4; ++r)
#pragma unroll
      for (int k = 0; k < 8; ++k) x[k] = __builtin_amdgcn_exp2f(-x[k]);
  }
  float s = 0.f;
#pragma unroll
  for (int k = 0; k < 8; ++k) s += x[k];
  write_sink(sink, s);
}

// Four pairs per iteration, 8 pixels each (32 pixel-pairs per thread).
__global__ __launch_bounds__(kProbeThreads) void probe_fwd_body_kernel(int iters, float thr, float *sink) {
  const int lane = threadIdx.x & 63;
  const float px = float(lane & 15) + 0.5f;
  const float py = float((lane >> 4) * 8) + 0.5f;
  float ux[4], uy[4], c0[4], c1[4], c2[4], c22[4], w[4];
#pragma unroll
  for (int j = 0; j < 4; ++j) {
    // per-lane values, as the kernel's pair constants (read from LDS) are
    const float l = 1e-4f * float(lane);
    ux[j] = 7.f + 0.37f * float(j) + l;
    uy[j] = 9.f - 0.51f * float(j) - l;
    c0[j] = -0.05f - 0.01f * float(j) - l;
    c1[j] = 0.004f * float(j) + l;
    c2[j] = -0.04f - 0.005f * float(j) - l;
    c22[j] = 2.f * c2[j];
    w[j] = 0.1f + 0.01f * float(j) + l;
  }
  float acc[8];
#pragma unroll
  for (int k = 0; k < 8; ++k) acc[k] = 0.f;
  for (int it = 0; it < iters; ++it) {
#pragma unroll
    for (int j = 0; j < 4; ++j) {
      const float dx = px - ux[j];
      const float dy = py - uy[j];
      const float A = c0[j] * dx * dx;
      const float B = c1[j] * dx;
      const float arg0 = fmaf(dy, fmaf(c2[j], dy, B), A);
      const float E = fmaf(c22[j], dy, B);
#pragma unroll
      for (int k = 0; k < 8; ++k) {
        const float fk = float(k);
        const float arg = (k == 0) ? arg0 : fmaf(fk, fmaf(c2[j], fk, E), arg0);
        const float ex = __builtin_amdgcn_exp2f(arg);
        acc[k] = fmaf(w[j], (arg >= thr) ? ex : 0.f, acc[k]);
      }
    }
#pragma unroll
    for (int j = 0; j < 4; ++j) ux[j] += 1e-3f;
  }
  float s = 0.f;
#pragma unroll
  for (int k = 0; k < 8; ++k) s += acc[k];
  write_sink(sink, s);
}

// One pair per iteration over an 8 x 8 quadrant (64 pixel-pairs per thread).
__global__ __launch_bounds__(kProbeThreads) void probe_bwd_body_kernel(int iters, float thr, float *sink) {
  const int lane = threadIdx.x & 63;
  float G0[8], G1[8];
#pragma unroll
  for (int u = 0; u < 8; ++u) {
    G0[u] = 1e-3f * float((lane * 7 + u * 13) & 31) - 0.015f;
    G1[u] = G0[u] * (float(u) - 3.5f);
  }
  float qx = 0.3f + 0.01f * float(lane & 7), qy = -0.7f + 0.02f * float(lane >> 3);
  const float cx = -0.06f - 1e-4f * float(lane), cy = 0.01f + 1e-4f * float(lane), cz = -0.05f - 1e-4f * float(lane);
  float tot[6] = {0.f, 0.f, 0.f, 0.f, 0.f, 0.f};
  for (int it = 0; it < iters; ++it) {
    const float m2aqx = -2.f * cx * qx;
    const float aqx2 = cx * qx * qx;
    const float mbqx = -cy * qx;
    float A[8] = {0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f};
    float Sr = 0.f, Scr = 0.f, Srr = 0.f;
#pragma unroll 1
    for (int row = 0; row < 8; ++row) {
      const float rr = float(row) - 3.5f;
      const float dy = rr - qy;
      const float brow = fmaf(cy, dy, m2aqx);
      const float drow = fmaf(dy, fmaf(cz, dy, mbqx), aqx2);
      float R0 = 0.f, R1 = 0.f;
#pragma unroll
      for (int u = 0; u < 8; ++u) {
        const float cc = float(u) - 3.5f;
        const float arg = fmaf(cc, fmaf(cx, cc, brow), drow);
        const float ex = (arg >= thr) ? __builtin_amdgcn_exp2f(arg) : 0.f;
        A[u] = fmaf(G0[u], ex, A[u]);
        R0 = fmaf(G0[u], ex, R0);
        R1 = fmaf(G1[u], ex, R1);
      }
      Sr = fmaf(R0, rr, Sr);
      Scr = fmaf(R1, rr, Scr);
      Srr = fmaf(R0, rr * rr, Srr);
    }
    float S0 = 0.f, Sc = 0.f, Scc = 0.f;
#pragma unroll
    for (int col = 0; col < 8; ++col) {
      const float cc = float(col) - 3.5f;
      S0 += A[col];
      Sc = fmaf(A[col], cc, Sc);
      Scc = fmaf(A[col], cc * cc, Scc);
    }
    tot[0] += S0;
    tot[1] += fmaf(-qx, S0, Sc);
    tot[2] += fmaf(-qy, S0, Sr);
    tot[3] += fmaf(qx * qx, S0, fmaf(-2.f * qx, Sc, Scc));
    tot[4] += fmaf(qx * qy, S0, fmaf(-qy, Sc, fmaf(-qx, Sr, Scr)));
    tot[5] += fmaf(qy * qy, S0, fmaf(-2.f * qy, Sr, Srr));
    qx += 1e-3f;
    qy -= 1e-3f;
  }
  write_sink(sink, tot[0] + tot[1] + tot[2] + tot[3] + tot[4] + tot[5]);
}

// Each lane reads 8 float4 per iteration; the lanes of a wave read 64
// consecutive float4 (1 KiB), so no two lanes share a bank group.
__global__ __launch_bounds__(kProbeThreads) void probe_lds_kernel(int iters, float *sink) {
  __shared__ float4 s[kProbeThreads * 4];
  for (int i = threadIdx.x; i < kProbeThreads * 4; i += kProbeThreads)
    s[i] = make_float4(float(i), 1.f, 2.f, 3.f);
  __syncthreads();
  const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
  float4 a = make_float4(0.f, 0.f, 0.f, 0.f);
  for (int it = 0; it < iters; ++it) {
#pragma unroll
    for (int j = 0; j < 8; ++j) {
      const int idx = (((wave * 4 + j + it) & 15) << 6) | lane;
      const float4 v = s[idx];
      a.x += v.x;
      a.y += v.y;
      a.z += v.z;
      a.w += v.w;
    }
  }
  write_sink(sink, a.x + a.y + a.z + a.w);
}

__global__ __launch_bounds__(kProbeThreads) void probe_mfma_kernel(int iters, float *sink) {
  const int lane = threadIdx.x & 63;
  bf16x8 a, b;
#pragma unroll
  for (int k = 0; k < 8; ++k) {
    a[k] = __bf16(float((lane + k) & 7) * 0.125f);
    b[k] = __bf16(float((lane * 3 + k) & 7) * 0.0625f);
  }
  f32x16 acc[4];
#pragma unroll
  for (int t = 0; t < 4; ++t)
#pragma unroll
    for (int r = 0; r < 16; ++r) acc[t][r] = 0.f;
  for (int it = 0; it < iters; ++it) {
#pragma unroll
    for (int t = 0; t < 4; ++t) acc[t] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(a, b, acc[t], 0, 0, 0);
  }
  float s = 0.f;
#pragma unroll
  for (int t = 0; t < 4; ++t)
#pragma unroll
    for (int r = 0; r < 16; ++r) s += acc[t][r];
  write_sink(sink, s);
}

}  // namespace
}  // namespace fgs

using namespace fgs;

extern "C" int fgs_probe(int32_t kind, int32_t blocks, int32_t iters, float *sink, double *work,
                         void *stream) {
  if (blocks <= 0 || iters <= 0 || !sink || !work) return fail(FGS_E_INVALID, "probe: blocks, iters > 0, sink, work");
  hipStream_t s = static_cast<hipStream_t>(stream);
  const double threads = double(blocks) * kProbeThreads;
  const double waves = threads / 64.0;
  const float thr = -0.5f * kLog2e * 9.f;
  switch (kind) {
    case FGS_PROBE_FMA:
      probe_fma_kernel<<<blocks, kProbeThreads, 0, s>>>(iters, 0.999f, 1e-3f, sink);
      *work = threads * iters * 32.0 * 2.0;  // flops
      break;
    case FGS_PROBE_EXP:
      probe_exp_kernel<<<blocks, kProbeThreads, 0, s>>>(iters, sink);
      *work = threads * iters * 32.0;  // v_exp_f32 lane operations
      break;
    case FGS_PROBE_FWD_BODY:
      probe_fwd_body_kernel<<<blocks, kProbeThreads, 0, s>>>(iters, thr, sink);
      *work = threads * iters * 32.0;  // (pixel, Gaussian) pairs
      break;
    case FGS_PROBE_BWD_BODY:
      probe_bwd_body_kernel<<<blocks, kProbeThreads, 0, s>>>(iters, thr, sink);
      *work = threads * iters * 64.0;  // (pixel, Gaussian) pairs
      break;
    case FGS_PROBE_LDS:
      probe_lds_kernel<<<blocks, kProbeThreads, 0, s>>>(iters, sink);
      *work = threads * iters * 8.0 * 16.0;  // bytes read from LDS
      break;
    case FGS_PROBE_MFMA_BF16:
      probe_mfma_kernel<<<blocks, kProbeThreads, 0, s>>>(iters, sink);
      *work = waves * iters * 4.0 * (2.0 * 32 * 32 * 16);  // flops
      break;
    default:
      return fail(FGS_E_INVALID, "probe: unknown kind");
  }
  FGS_LAUNCH_CHECK("probe kernel");
  return FGS_OK;
}
