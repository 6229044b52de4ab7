// Learned initializer: a 3-layer MLP (544 -> 128 -> 128 -> 32 padded, 8
// used) mapping an 8^3 patch of the FDK volume plus the position to a
// Gaussian's density, log-scales and rotation. BF16 operands, FP32
// accumulation on the gfx950 matrix cores (v_mfma_f32_32x32x16_bf16).
//
// All matrices are row-major with the reduction index contiguous, and every
// product is an "NT" GEMM C[m][n] = sum_k A[m][k] B[n][k]:
//   forward   Z = X W^T + b                    A = X [M][K],     B = W [N][K]
//   dX        dH = dZ W                         A = dZ [M][N],    B = W^T [K][N]
//   dW        dW = dZ^T X                       A = dZ^T [N][M],  B = X^T [K][M]
// so the forward also writes transposed activations and the backward
// transposed gradients (batch contiguous) for the weight products.
// Operand fragments are 16-byte loads straight from memory: lane l of a wave
// holds row l % 32, reduction slots 8 (l / 32) .. +7 of A and of B; the
// 32x32 FP32 result sits in 16 registers per lane, register r holding row
// 8 (r / 4) + 4 (l / 32) + r % 4, column l % 32.
// BF16 is round-to-nearest-even from FP32.
#include <algorithm>
#include <cmath>

#include "fgs_internal.h"

namespace fgs {
namespace {

typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef short i16x8 __attribute__((ext_vector_type(8)));
typedef float f32x16 __attribute__((ext_vector_type(16)));

__device__ __forceinline__ uint16_t to_bf16(float f) {
  uint32_t u = __float_as_uint(f);
  if ((u & 0x7fffffffu) > 0x7f800000u) return uint16_t((u >> 16) | 0x40u);  // NaN stays NaN
  u += 0x7fffu + ((u >> 16) & 1u);
  return uint16_t(u >> 16);
}

__device__ __forceinline__ float from_bf16(uint16_t h) { return __uint_as_float(uint32_t(h) << 16); }

__device__ __forceinline__ bf16x8 load8(const uint16_t *p) {
  const i16x8 v = *reinterpret_cast<const i16x8 *>(p);
  return __builtin_bit_cast(bf16x8, v);
}

enum Epi { kEpiFwd = 0, kEpiData = 1, kEpiWeight = 2 };

struct EpiArgs {
  const float *bias;    // fwd: [N]
  int relu;             // fwd: apply ReLU to H
  float *Z;             // fwd: pre-activation [M][N] (FP32)
  uint16_t *H;          // fwd: activation [M][N] (BF16) or null
  uint16_t *Ht;         // fwd: activation transposed [N][M] or null
  const float *mask_z;  // data: pre-activation of the layer below [M][N]; null = no ReLU
  uint16_t *D;          // data: gradient [M][N] (BF16)
  uint16_t *Dt;         // data: gradient transposed [N][M]
  float *C;             // weight: [M][N] (FP32)
};

constexpr int kNT = 4;  // 32-wide column tiles per wave

template <int EPI>
__global__ __launch_bounds__(256) void gemm_nt_kernel(const uint16_t *__restrict__ A,
                                                      const uint16_t *__restrict__ B, int M, int N, int K,
                                                      int kchunk, EpiArgs e) {
  const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
  const int m0 = (blockIdx.x * 4 + wave) * 32;
  const int n0 = blockIdx.y * 32 * kNT;
  if (m0 >= M) return;
  const int kofs = 8 * (lane >> 5);
  const uint16_t *arow = A + int64_t(m0 + (lane & 31)) * K + kofs;
  f32x16 acc[kNT];
#pragma unroll
  for (int t = 0; t < kNT; ++t)
#pragma unroll
    for (int r = 0; r < 16; ++r) acc[t][r] = 0.f;
  const i16x8 zero8 = {0, 0, 0, 0, 0, 0, 0, 0};
  // split-K (weight products): slice blockIdx.z covers [kb, ke) and writes
  // its own partial product
  const int kb = blockIdx.z * kchunk, ke = min(K, kb + kchunk);
  for (int k = kb; k < ke; k += 16) {
    const bf16x8 a = load8(arow + k);
#pragma unroll
    for (int t = 0; t < kNT; ++t) {
      const int col = n0 + 32 * t + (lane & 31);
      const bf16x8 b = (col < N) ? load8(B + int64_t(col) * K + kofs + k) : __builtin_bit_cast(bf16x8, zero8);
      acc[t] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(a, b, acc[t], 0, 0, 0);
    }
  }
#pragma unroll
  for (int t = 0; t < kNT; ++t) {
    const int col = n0 + 32 * t + (lane & 31);
    if (col >= N) continue;
#pragma unroll
    for (int r = 0; r < 16; ++r) {
      const int row = m0 + 8 * (r >> 2) + 4 * (lane >> 5) + (r & 3);
      const int64_t o = int64_t(row) * N + col;
      float v = acc[t][r];
      if (EPI == kEpiFwd) {
        v += e.bias[col];
        e.Z[o] = v;
        const float h = e.relu ? fmaxf(v, 0.f) : v;
        const uint16_t hb = to_bf16(h);
        if (e.H) e.H[o] = hb;
        if (e.Ht) e.Ht[int64_t(col) * M + row] = hb;
      } else if (EPI == kEpiData) {
        if (e.mask_z && !(e.mask_z[o] > 0.f)) v = 0.f;
        const uint16_t db = to_bf16(v);
        e.D[o] = db;
        e.Dt[int64_t(col) * M + row] = db;
      } else {
        e.C[int64_t(blockIdx.z) * M * N + o] = v;
      }
    }
  }
}

// Reduction slices of a weight product: enough workgroups to fill the chip,
// each slice at least kMinChunk deep.
constexpr int kMinChunk = 512;
constexpr int kMaxSplit = 128;

inline int split_count(int M, int N, int K) {
  const int tiles = ((M / 32 + 3) / 4) * ((N + 32 * kNT - 1) / (32 * kNT));
  int s = (1024 + tiles - 1) / tiles;
  s = std::min(s, std::max(1, K / kMinChunk));
  return std::max(1, std::min(s, kMaxSplit));
}

inline int chunk_for(int K, int splits) { return ((K + splits - 1) / splits + 15) / 16 * 16; }

template <int EPI>
int gemm_nt(const uint16_t *A, const uint16_t *B, int M, int N, int K, const EpiArgs &e, hipStream_t s,
            int splits = 1) {
  if (M % 32 || N % 32 || K % 16 || M <= 0 || N <= 0 || K <= 0)
    return fail(FGS_E_INVALID, "GEMM sizes must be multiples of 32 (rows, columns) and 16 (reduction)");
  const int kchunk = chunk_for(K, splits);
  dim3 grid(unsigned((M / 32 + 3) / 4), unsigned((N + 32 * kNT - 1) / (32 * kNT)), unsigned(splits));
  gemm_nt_kernel<EPI><<<grid, 256, 0, s>>>(A, B, M, N, K, kchunk, e);
  FGS_LAUNCH_CHECK("gemm_nt_kernel");
  return FGS_OK;
}

// C[i] = sum over slices z (in order) of P[z][i].
__global__ __launch_bounds__(256) void split_sum_kernel(const float *__restrict__ P, int splits, int64_t len,
                                                        float *__restrict__ C) {
  const int64_t i = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (i >= len) return;
  float acc = 0.f;
  for (int z = 0; z < splits; ++z) acc += P[int64_t(z) * len + i];
  C[i] = acc;
}

// Weight gradient C[M][N] = A B^T over a long reduction, split into slices
// whose partial products go to `part` and are summed in a fixed order.
int weight_grad(const uint16_t *A, const uint16_t *B, int M, int N, int K, float *C, float *part, hipStream_t s) {
  const int splits = split_count(M, N, K);
  EpiArgs e{};
  e.C = splits > 1 ? part : C;
  int st = gemm_nt<kEpiWeight>(A, B, M, N, K, e, s, splits);
  if (st != FGS_OK || splits == 1) return st;
  const int64_t len = int64_t(M) * N;
  split_sum_kernel<<<grid_for(uint64_t(len), 256), 256, 0, s>>>(part, splits, len, C);
  FGS_LAUNCH_CHECK("split_sum_kernel");
  return FGS_OK;
}

// db[n] = sum over m of D^T[n][m] (BF16 gradients), one block per row.
__global__ __launch_bounds__(256) void row_sum_kernel(const uint16_t *__restrict__ Dt, int M, float *__restrict__ db) {
  __shared__ float sh[4];
  const uint16_t *row = Dt + int64_t(blockIdx.x) * M;
  float acc = 0.f;
  for (int m = threadIdx.x; m < M; m += 256) acc += from_bf16(row[m]);
  for (int d = 32; d > 0; d >>= 1) acc += __shfl_xor(acc, d, 64);
  if ((threadIdx.x & 63) == 0) sh[threadIdx.x >> 6] = acc;
  __syncthreads();
  if (threadIdx.x == 0) db[blockIdx.x] = (sh[0] + sh[1]) + (sh[2] + sh[3]);
}

__global__ __launch_bounds__(256) void pack_kernel(const float *__restrict__ W, int N, int K, uint16_t *__restrict__ Wb,
                                                   uint16_t *__restrict__ Wbt) {
  const int64_t i = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (i >= int64_t(N) * K) return;
  const int n = int(i / K), k = int(i % K);
  const uint16_t h = to_bf16(W[i]);
  Wb[i] = h;
  if (Wbt) Wbt[int64_t(k) * N + n] = h;
}

// Patch features: 8^3 trilinear samples of vol, one voxel apart, centred on
// the Gaussian's mean, times inv_norm; then the mean scaled to [-1, 1]
// (x 2); zero padding to kFeat. One 256-thread block per row (sample).
constexpr int kPatch = 8;
constexpr int kFeat = 544;

struct PatchGrid {
  float origin[3], h[3];
  int dims[3];
};

__device__ __forceinline__ float trilinear_at(const float *__restrict__ vol, const PatchGrid &G, float cx, float cy,
                                              float cz) {
  const float fx = floorf(cx), fy = floorf(cy), fz = floorf(cz);
  const int x0 = int(fx), y0 = int(fy), z0 = int(fz);
  const float a = cx - fx, b = cy - fy, g = cz - fz;
  float acc = 0.f;
  for (int dz = 0; dz < 2; ++dz)
    for (int dy = 0; dy < 2; ++dy)
      for (int dx = 0; dx < 2; ++dx) {
        const int x = x0 + dx, y = y0 + dy, z = z0 + dz;
        if (x < 0 || x >= G.dims[0] || y < 0 || y >= G.dims[1] || z < 0 || z >= G.dims[2]) continue;
        const float w = (dx ? a : 1.f - a) * (dy ? b : 1.f - b) * (dz ? g : 1.f - g);
        acc = fmaf(w, vol[(int64_t(z) * G.dims[1] + y) * G.dims[0] + x], acc);
      }
  return acc;
}

__global__ __launch_bounds__(256) void gather_kernel(const float *__restrict__ vol, PatchGrid G, float inv_norm,
                                                     const float *__restrict__ norm_max,
                                                     const float *__restrict__ mean,
                                                     const float *__restrict__ extra, int n_extra, int64_t n,
                                                     int rows, uint16_t *__restrict__ X,
                                                     uint16_t *__restrict__ Xt) {
  const int m = blockIdx.x;
  const bool valid = m < n;
  if (norm_max) inv_norm = inv_norm / norm_max[0];
  float c[3] = {0.f, 0.f, 0.f}, p[3] = {0.f, 0.f, 0.f};
  if (valid)
    for (int a = 0; a < 3; ++a) {
      p[a] = mean[a * n + m];
      c[a] = (p[a] - G.origin[a]) / G.h[a] - 0.5f;
    }
  for (int f = threadIdx.x; f < kFeat; f += blockDim.x) {
    float v = 0.f;
    if (valid) {
      if (f < kPatch * kPatch * kPatch) {
        const int ix = f & 7, iy = (f >> 3) & 7, iz = f >> 6;
        v = inv_norm * trilinear_at(vol, G, c[0] + float(ix) - 3.5f, c[1] + float(iy) - 3.5f,
                                    c[2] + float(iz) - 3.5f);
      } else if (f < kPatch * kPatch * kPatch + 3) {
        v = 2.f * p[f - kPatch * kPatch * kPatch];
      } else if (f < kPatch * kPatch * kPatch + 3 + n_extra) {
        v = extra[int64_t(f - kPatch * kPatch * kPatch - 3) * n + m];
      }
    }
    const uint16_t h = to_bf16(v);
    X[int64_t(m) * kFeat + f] = h;
    if (Xt) Xt[int64_t(f) * rows + m] = h;
  }
}

// A fitted Gaussian whose density is at most this carries no shape
// information: its scale and rotation terms are left out of the loss.
constexpr float kLiveDensity = 1e-3f;

// Prediction heads and loss. y = Z3 row (8 used of ld): density = softplus(y0),
// log-scales base + y1..y3 (base = per-sample offset, or 0), rotation =
// (y4..y7) / |.|. Training loss per sample (rho - rho_t)^2 + live *
// (|s - s_t|^2 + (1 - (q . q_t)^2)), live = [rho_t > kLiveDensity],
// averaged over n.
__global__ __launch_bounds__(256) void heads_kernel(const float *__restrict__ Z3, int ld, int64_t n, int rows,
                                                    const float *__restrict__ base_ls,
                                                    const float *__restrict__ target, float *__restrict__ out,
                                                    uint16_t *__restrict__ D, uint16_t *__restrict__ Dt,
                                                    float *__restrict__ partial) {
  __shared__ float sh[4];
  const int64_t m = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  float lm = 0.f;
  float g[8] = {0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f};
  if (m < n) {
    const float *y = Z3 + m * ld;
    const float y0 = y[0];
    const float rho = (y0 > 20.f) ? y0 : log1pf(expf(y0));
    const float sig = 1.f / (1.f + expf(-y0));
    float q[4] = {y[4], y[5], y[6], y[7]};
    const float qn = fmaxf(sqrtf(q[0] * q[0] + q[1] * q[1] + q[2] * q[2] + q[3] * q[3]), 1e-12f);
    float qh[4];
    for (int j = 0; j < 4; ++j) qh[j] = q[j] / qn;
    const float base = base_ls ? base_ls[m] : 0.f;
    float ls[3];
    for (int j = 0; j < 3; ++j) ls[j] = base + y[1 + j];
    if (out) {
      out[m] = rho;
      for (int j = 0; j < 3; ++j) out[(1 + j) * n + m] = ls[j];
      for (int j = 0; j < 4; ++j) out[(4 + j) * n + m] = qh[j];
    }
    if (target) {
      const float *t = target + m * 8;
      const float inv_n = 1.f / float(n);
      const float dr = rho - t[0];
      float l = dr * dr;
      g[0] = 2.f * dr * sig * inv_n;
      if (t[0] > kLiveDensity) {
        for (int j = 0; j < 3; ++j) {
          const float ds = ls[j] - t[1 + j];
          l += ds * ds;
          g[1 + j] = 2.f * ds * inv_n;
        }
        const float dot = qh[0] * t[4] + qh[1] * t[5] + qh[2] * t[6] + qh[3] * t[7];
        l += 1.f - dot * dot;
        // d/dqh of -(qh . t)^2 = -2 dot t, projected through the normalisation
        float gh[4], proj = 0.f;
        for (int j = 0; j < 4; ++j) {
          gh[j] = -2.f * dot * t[4 + j];
          proj += gh[j] * qh[j];
        }
        for (int j = 0; j < 4; ++j) g[4 + j] = (gh[j] - qh[j] * proj) / qn * inv_n;
      }
      lm = l;
    }
  }
  if (D && m < rows) {
    for (int j = 0; j < ld; ++j) {
      const uint16_t h = to_bf16(j < 8 ? g[j] : 0.f);
      D[m * ld + j] = h;
      Dt[int64_t(j) * rows + m] = h;
    }
  }
  if (partial) {
    const float t = block_sum_f32<256>(lm, sh);
    if (threadIdx.x == 0) partial[blockIdx.x] = t;
  }
}

__global__ __launch_bounds__(256) void loss_final_kernel(const float *__restrict__ partial, int nb, float inv_n,
                                                         float *__restrict__ loss) {
  __shared__ float sh[4];
  CompSum acc;
  for (int i = threadIdx.x; i < nb; i += 256) acc.add(partial[i]);
  const float t = block_sum_f32<256>(acc.value(), sh);
  if (threadIdx.x == 0) loss[0] = t * inv_n;
}

int check_net(const fgs_mlp *net) {
  if (!net || !net->w1 || !net->w1t || !net->w2 || !net->w2t || !net->w3 || !net->w3t || !net->b1 || !net->b2 ||
      !net->b3)
    return fail(FGS_E_INVALID, "null network pointer");
  if (net->k_in != kFeat || net->hidden != 128 || net->n_out != 32)
    return fail(FGS_E_UNSUPPORTED, "network shape must be 544 -> 128 -> 128 -> 32");
  return FGS_OK;
}

}  // namespace
}  // namespace fgs

using namespace fgs;

extern "C" int fgs_gather_patches(const float *vol, const fgs_grid *grid, float inv_norm, const float *norm_max,
                                  const float *mean, const float *extra, int32_t n_extra, int64_t n, int32_t rows,
                                  uint16_t *x, uint16_t *xt, void *stream) {
  if (!vol || !grid || !mean || !x) return fail(FGS_E_INVALID, "null argument");
  if (n_extra < 0 || n_extra > kFeat - kPatch * kPatch * kPatch - 3 || (n_extra > 0 && !extra))
    return fail(FGS_E_INVALID, "extra features: 0..29 rows of n values");
  if (n <= 0 || rows < n || rows % 32) return fail(FGS_E_INVALID, "rows must be >= n and a multiple of 32");
  PatchGrid G{};
  for (int a = 0; a < 3; ++a) {
    if (grid->dims[a] <= 0 || !(grid->spacing[a] > 0.f)) return fail(FGS_E_INVALID, "grid");
    G.origin[a] = grid->origin[a];
    G.h[a] = grid->spacing[a];
    G.dims[a] = grid->dims[a];
  }
  hipStream_t s = static_cast<hipStream_t>(stream);
  gather_kernel<<<unsigned(rows), 256, 0, s>>>(vol, G, inv_norm, norm_max, mean, extra, n_extra, n, rows, x,
                                                  xt);
  FGS_LAUNCH_CHECK("gather_kernel");
  return FGS_OK;
}

extern "C" int fgs_mlp_pack(const float *w, int32_t n_out, int32_t k_in, uint16_t *wb, uint16_t *wbt, void *stream) {
  if (!w || !wb || n_out <= 0 || k_in <= 0) return fail(FGS_E_INVALID, "invalid argument");
  hipStream_t s = static_cast<hipStream_t>(stream);
  pack_kernel<<<grid_for(uint64_t(n_out) * k_in, 256), 256, 0, s>>>(w, n_out, k_in, wb, wbt);
  FGS_LAUNCH_CHECK("pack_kernel");
  return FGS_OK;
}

extern "C" int fgs_mlp_fwd(const fgs_mlp *net, const uint16_t *x, int32_t rows, fgs_mlp_acts *acts, void *stream) {
  int st = check_net(net);
  if (st != FGS_OK) return st;
  if (!x || !acts || !acts->z1 || !acts->z2 || !acts->z3 || !acts->h1 || !acts->h2)
    return fail(FGS_E_INVALID, "null activation buffer");
  hipStream_t s = static_cast<hipStream_t>(stream);
  EpiArgs e{};
  e.bias = net->b1; e.relu = 1; e.Z = acts->z1; e.H = acts->h1; e.Ht = acts->h1t;
  st = gemm_nt<kEpiFwd>(x, net->w1, rows, net->hidden, net->k_in, e, s);
  if (st != FGS_OK) return st;
  e = EpiArgs{};
  e.bias = net->b2; e.relu = 1; e.Z = acts->z2; e.H = acts->h2; e.Ht = acts->h2t;
  st = gemm_nt<kEpiFwd>(acts->h1, net->w2, rows, net->hidden, net->hidden, e, s);
  if (st != FGS_OK) return st;
  e = EpiArgs{};
  e.bias = net->b3; e.relu = 0; e.Z = acts->z3;
  return gemm_nt<kEpiFwd>(acts->h2, net->w3, rows, net->n_out, net->hidden, e, s);
}

extern "C" int fgs_mlp_heads(const float *z3, int32_t rows, int64_t n, const float *base_log_scale,
                             const float *target, float *params_out,
                             uint16_t *dz3, uint16_t *dz3t, float *loss, fgs_workspace *ws, void *stream) {
  if (!z3 || n <= 0 || rows < n || rows % 32) return fail(FGS_E_INVALID, "invalid sizes");
  if (target && (!dz3 || !dz3t || !loss || !ws || !ws->ptr)) return fail(FGS_E_INVALID, "training needs gradient, loss and workspace");
  hipStream_t s = static_cast<hipStream_t>(stream);
  const int nb = int((uint64_t(rows) + 255) / 256);
  float *partial = nullptr;
  if (target) {
    ws->needed = uint64_t(nb) * sizeof(float);
    if (ws->bytes < ws->needed) return fail(FGS_E_CAPACITY, "workspace too small");
    partial = static_cast<float *>(ws->ptr);
  }
  heads_kernel<<<nb, 256, 0, s>>>(z3, 32, n, rows, base_log_scale, target, params_out, target ? dz3 : nullptr,
                                  dz3t, partial);
  FGS_LAUNCH_CHECK("heads_kernel");
  if (target) {
    loss_final_kernel<<<1, 256, 0, s>>>(partial, nb, float(1.0 / double(n)), loss);
    FGS_LAUNCH_CHECK("loss_final_kernel");
  }
  return FGS_OK;
}

extern "C" int fgs_mlp_bwd(const fgs_mlp *net, const uint16_t *xt, int32_t rows, const fgs_mlp_acts *acts,
                           const uint16_t *dz3, const uint16_t *dz3t, fgs_mlp_grads *grads, fgs_workspace *ws,
                           void *stream) {
  int st = check_net(net);
  if (st != FGS_OK) return st;
  if (!xt || !acts || !acts->h1t || !acts->h2t || !dz3 || !dz3t || !grads || !ws)
    return fail(FGS_E_INVALID, "null argument");
  const int H = net->hidden;
  Carver c(nullptr);
  uint64_t o2, o2t, o1, o1t;
  c.take<uint16_t>(uint64_t(rows) * H, &o2);
  c.take<uint16_t>(uint64_t(rows) * H, &o2t);
  c.take<uint16_t>(uint64_t(rows) * H, &o1);
  c.take<uint16_t>(uint64_t(rows) * H, &o1t);
  uint64_t op;
  const int s1 = split_count(H, net->k_in, rows), s2 = split_count(H, H, rows), s3 = split_count(net->n_out, H, rows);
  const uint64_t part = std::max({uint64_t(s1) * H * net->k_in, uint64_t(s2) * H * H, uint64_t(s3) * net->n_out * H});
  c.take<float>(part, &op);
  ws->needed = c.used;
  if (!ws->ptr || ws->bytes < ws->needed) return fail(FGS_E_CAPACITY, "workspace too small");
  char *b = static_cast<char *>(ws->ptr);
  uint16_t *dz2 = reinterpret_cast<uint16_t *>(b + o2), *dz2t = reinterpret_cast<uint16_t *>(b + o2t);
  uint16_t *dz1 = reinterpret_cast<uint16_t *>(b + o1), *dz1t = reinterpret_cast<uint16_t *>(b + o1t);
  float *pbuf = reinterpret_cast<float *>(b + op);
  hipStream_t s = static_cast<hipStream_t>(stream);
  // layer 3
  st = weight_grad(dz3t, acts->h2t, net->n_out, H, rows, grads->dw3, pbuf, s);
  if (st != FGS_OK) return st;
  row_sum_kernel<<<net->n_out, 256, 0, s>>>(dz3t, rows, grads->db3);
  EpiArgs e{};
  e.mask_z = acts->z2; e.D = dz2; e.Dt = dz2t;
  st = gemm_nt<kEpiData>(dz3, net->w3t, rows, H, net->n_out, e, s);
  if (st != FGS_OK) return st;
  // layer 2
  st = weight_grad(dz2t, acts->h1t, H, H, rows, grads->dw2, pbuf, s);
  if (st != FGS_OK) return st;
  row_sum_kernel<<<H, 256, 0, s>>>(dz2t, rows, grads->db2);
  e = EpiArgs{};
  e.mask_z = acts->z1; e.D = dz1; e.Dt = dz1t;
  st = gemm_nt<kEpiData>(dz2, net->w2t, rows, H, H, e, s);
  if (st != FGS_OK) return st;
  // layer 1
  st = weight_grad(dz1t, xt, H, net->k_in, rows, grads->dw1, pbuf, s);
  if (st != FGS_OK) return st;
  row_sum_kernel<<<H, 256, 0, s>>>(dz1t, rows, grads->db1);
  FGS_LAUNCH_CHECK("row_sum_kernel");
  return FGS_OK;
}

namespace fgs {
namespace {

// Quaternion (w, x, y, z) of a proper rotation matrix (Shepperd's method:
// branch on the largest of the trace and the diagonal for stability).
__device__ void rot_to_quat(const float R[9], float q[4]) {
  const float tr = R[0] + R[4] + R[8];
  if (tr >= R[0] && tr >= R[4] && tr >= R[8]) {
    const float s = sqrtf(fmaxf(1.f + tr, 0.f)) * 2.f;
    q[0] = 0.25f * s;
    q[1] = (R[7] - R[5]) / s;
    q[2] = (R[2] - R[6]) / s;
    q[3] = (R[3] - R[1]) / s;
  } else if (R[0] >= R[4] && R[0] >= R[8]) {
    const float s = sqrtf(fmaxf(1.f + R[0] - R[4] - R[8], 0.f)) * 2.f;
    q[0] = (R[7] - R[5]) / s;
    q[1] = 0.25f * s;
    q[2] = (R[1] + R[3]) / s;
    q[3] = (R[2] + R[6]) / s;
  } else if (R[4] >= R[8]) {
    const float s = sqrtf(fmaxf(1.f + R[4] - R[0] - R[8], 0.f)) * 2.f;
    q[0] = (R[2] - R[6]) / s;
    q[1] = (R[1] + R[3]) / s;
    q[2] = 0.25f * s;
    q[3] = (R[5] + R[7]) / s;
  } else {
    const float s = sqrtf(fmaxf(1.f + R[8] - R[0] - R[4], 0.f)) * 2.f;
    q[0] = (R[3] - R[1]) / s;
    q[1] = (R[2] + R[6]) / s;
    q[2] = (R[5] + R[7]) / s;
    q[3] = 0.25f * s;
  }
  if (q[0] < 0.f)
    for (int j = 0; j < 4; ++j) q[j] = -q[j];
}

__global__ __launch_bounds__(256) void canonical_kernel(fgs_gaussians g, float *__restrict__ out) {
  const int64_t i = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (i >= g.n) return;
  GaussParams P;
  load_gauss(g, i, P);
  const int64_t n = g.n;
  float ls[3] = {g.log_scale[i], g.log_scale[n + i], g.log_scale[2 * n + i]};
  // stable descending order of the three log-scales
  int o[3] = {0, 1, 2};
  for (int a = 0; a < 2; ++a)
    for (int b = 0; b < 2 - a; ++b)
      if (ls[o[b + 1]] > ls[o[b]]) {
        const int t = o[b];
        o[b] = o[b + 1];
        o[b + 1] = t;
      }
  float R[9];
  for (int r = 0; r < 3; ++r)
    for (int c = 0; c < 3; ++c) R[3 * r + c] = P.R[3 * r + o[c]];
  const float det = R[0] * (R[4] * R[8] - R[5] * R[7]) - R[1] * (R[3] * R[8] - R[5] * R[6]) +
                    R[2] * (R[3] * R[7] - R[4] * R[6]);
  if (det < 0.f)
    for (int r = 0; r < 3; ++r) R[3 * r + 2] = -R[3 * r + 2];
  float q[4];
  rot_to_quat(R, q);
  float *t = out + i * 8;
  t[0] = P.rho;
  for (int j = 0; j < 3; ++j) t[1 + j] = ls[o[j]];
  for (int j = 0; j < 4; ++j) t[4 + j] = q[j];
}

}  // namespace
}  // namespace fgs

extern "C" int fgs_canonical_targets(const fgs_gaussians *g, float *out, void *stream) {
  if (!g || !out || g->n <= 0 || !g->log_scale || !g->quat || !g->density || !g->mean)
    return fail(FGS_E_INVALID, "invalid argument");
  hipStream_t s = static_cast<hipStream_t>(stream);
  canonical_kernel<<<grid_for(uint64_t(g->n), 256), 256, 0, s>>>(*g, out);
  FGS_LAUNCH_CHECK("canonical_kernel");
  return FGS_OK;
}
