// Adaptive density control (Sec. 3.4: the loss gradient is used to prune,
// clone or split Gaussians; Suppl. C: the count is capped 10% above the
// initial one) for gfx950.
//
//   accumulate   per optimiser step: stat[0][i] += |dL/dmean_i|,
//                stat[1][i] += [|dL/dmean_i| > 0]
//   densify      classify every Gaussian (prune / keep / clone / split) from
//                its mean accumulated gradient and its size; if the densify
//                candidates do not fit under the cap, a stable radix sort on
//                the score keeps the largest ones (ties: lower index); an
//                exclusive scan of the output counts gives every survivor
//                its place, and one kernel writes the new parameters and Adam
//                moments.
// All decisions are FP32 comparisons of FP32 values (scores by correctly
// rounded division, sizes in the log domain), so they are reproducible
// exactly on any implementation that takes them in FP32.
#include <cmath>

#include "fgs_internal.h"

namespace fgs {
namespace {

enum : uint32_t { kPrune = 0, kKeep = 1, kClone = 2, kSplit = 3 };

__global__ __launch_bounds__(256) void adc_accumulate_kernel(const float *__restrict__ gm, int64_t n,
                                                             float *__restrict__ stat) {
  const int64_t i = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const float x = gm[i], y = gm[n + i], z = gm[2 * n + i];
  const float norm = sqrtf(x * x + y * y + z * z);
  stat[i] += norm;
  stat[n + i] += (norm > 0.f) ? 1.f : 0.f;
}

__global__ void adc_zero_kernel(unsigned long long *p) {
  if (threadIdx.x < 2) p[threadIdx.x] = 0ull;
}

struct AdcThresholds {
  float grad;        // candidates: score > grad
  float ls_split;    // split when the largest log-scale > ls_split, else clone
  float rho_prune;   // prune when density < rho_prune
  float ls_prune;    // or the largest log-scale > ls_prune
};

// code[i]: kPrune, kKeep, or (for densify candidates) kClone / kSplit.
// key[i]: candidates ~bits(score) (descending score sorts first), others
// 0xffffffff; val[i] = i. counts[0] += survivors, counts[1] += candidates.
__global__ __launch_bounds__(256) void adc_classify_kernel(fgs_gaussians g, const float *__restrict__ stat,
                                                           AdcThresholds th, uint32_t *__restrict__ code,
                                                           uint32_t *__restrict__ key, uint32_t *__restrict__ val,
                                                           unsigned long long *__restrict__ counts) {
  const int64_t n = g.n;
  const int64_t i = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  uint32_t surv = 0, cand = 0;
  if (i < n) {
    const float ls = fmaxf(fmaxf(g.log_scale[i], g.log_scale[n + i]), g.log_scale[2 * n + i]);
    const float rho = g.density[i];
    const bool prune = !(rho >= th.rho_prune) || !(ls <= th.ls_prune);
    const float score = stat[i] / fmaxf(stat[n + i], 1.f);
    const bool c = !prune && score > th.grad;
    surv = prune ? 0u : 1u;
    cand = c ? 1u : 0u;
    code[i] = prune ? kPrune : (c ? (ls > th.ls_split ? kSplit : kClone) : kKeep);
    key[i] = c ? ~__float_as_uint(score) : 0xffffffffu;
    val[i] = uint32_t(i);
  }
  unsigned long long s = surv, c = cand;
  for (int d = 32; d > 0; d >>= 1) {
    s += __shfl_xor(s, d, 64);
    c += __shfl_xor(c, d, 64);
  }
  if ((threadIdx.x & 63) == 0) {
    if (s) atomicAdd(counts, s);
    if (c) atomicAdd(counts + 1, c);
  }
}

// Candidates ranked at or after `room` (by descending score, stable) stay as they are.
__global__ __launch_bounds__(256) void adc_demote_kernel(const uint32_t *__restrict__ sorted_vals, uint64_t room,
                                                         uint64_t n_cand, uint32_t *__restrict__ code) {
  const uint64_t k = room + uint64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (k >= n_cand) return;
  code[sorted_vals[k]] = kKeep;
}

__global__ __launch_bounds__(256) void adc_count_kernel(const uint32_t *__restrict__ code, int64_t n,
                                                        uint32_t *__restrict__ cnt) {
  const int64_t i = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const uint32_t c = code[i];
  cnt[i] = (c == kPrune) ? 0u : (c == kKeep ? 1u : 2u);
}

struct AdcOut {
  fgs_gaussians_out g;
  fgs_gaussian_grads m, v;
  int64_t n;
};

__device__ __forceinline__ void adc_put(const AdcOut &o, int64_t q, const float mean[3], const float ls[3],
                                        const float qt[4], float rho) {
  const int64_t n = o.n;
  for (int a = 0; a < 3; ++a) {
    o.g.mean[a * n + q] = mean[a];
    o.g.log_scale[a * n + q] = ls[a];
  }
  for (int a = 0; a < 4; ++a) o.g.quat[a * n + q] = qt[a];
  o.g.density[q] = rho;
}

__device__ __forceinline__ void adc_moments(const AdcOut &o, int64_t q, const fgs_gaussian_grads &m,
                                            const fgs_gaussian_grads &v, int64_t n_in, int64_t i) {
  const int64_t n = o.n;
  for (int a = 0; a < 3; ++a) {
    o.m.mean[a * n + q] = m.mean[a * n_in + i];
    o.v.mean[a * n + q] = v.mean[a * n_in + i];
    o.m.log_scale[a * n + q] = m.log_scale[a * n_in + i];
    o.v.log_scale[a * n + q] = v.log_scale[a * n_in + i];
  }
  for (int a = 0; a < 4; ++a) {
    o.m.quat[a * n + q] = m.quat[a * n_in + i];
    o.v.quat[a * n + q] = v.quat[a * n_in + i];
  }
  o.m.density[q] = m.density[i];
  o.v.density[q] = v.density[i];
}

// Kept: copied with its moments. Clone: the original and a copy, both at
// half density. Split: two children at mean + R diag(s) z (z the given
// standard normals), standard deviations divided by the shrink factor,
// density scaled so the pair carries the parent's mass. New Gaussians take
// their parent's Adam moments: with fresh (zero) moments late in a run, the
// step-count bias correction no longer compensates and their first few
// hundred updates would be several times the learning rate.
__global__ __launch_bounds__(256) void adc_emit_kernel(fgs_gaussians g, fgs_gaussian_grads m, fgs_gaussian_grads v,
                                                       const uint32_t *__restrict__ code,
                                                       const uint32_t *__restrict__ pos,
                                                       const float *__restrict__ normals, float ls_shrink,
                                                       float split_rho, AdcOut o) {
  const int64_t n = g.n;
  const int64_t i = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const uint32_t c = code[i];
  if (c == kPrune) return;
  const int64_t q = pos[i];
  float mean[3], ls[3], qt[4];
  for (int a = 0; a < 3; ++a) {
    mean[a] = g.mean[a * n + i];
    ls[a] = g.log_scale[a * n + i];
  }
  for (int a = 0; a < 4; ++a) qt[a] = g.quat[a * n + i];
  const float rho = g.density[i];
  if (c == kKeep) {
    adc_put(o, q, mean, ls, qt, rho);
    adc_moments(o, q, m, v, n, i);
    return;
  }
  if (c == kClone) {
    adc_put(o, q, mean, ls, qt, 0.5f * rho);
    adc_moments(o, q, m, v, n, i);
    adc_put(o, q + 1, mean, ls, qt, 0.5f * rho);
    adc_moments(o, q + 1, m, v, n, i);
    return;
  }
  GaussParams P;
  load_gauss(g, i, P);
  float cls[3];
  for (int a = 0; a < 3; ++a) cls[a] = ls[a] - ls_shrink;
  for (int child = 0; child < 2; ++child) {
    float z[3], cm[3];
    for (int j = 0; j < 3; ++j) z[j] = normals[(3 * child + j) * n + i] * P.s[j];
    for (int a = 0; a < 3; ++a) cm[a] = mean[a] + P.R[3 * a] * z[0] + P.R[3 * a + 1] * z[1] + P.R[3 * a + 2] * z[2];
    adc_put(o, q + child, cm, cls, qt, split_rho * rho);
    adc_moments(o, q + child, m, v, n, i);
  }
}

}  // namespace
}  // namespace fgs

using namespace fgs;

extern "C" int fgs_adc_accumulate(const float *grad_mean, int64_t n, float *stat, void *stream) {
  if (!grad_mean || !stat) return fail(FGS_E_INVALID, "null argument");
  if (n <= 0) return fail(FGS_E_INVALID, "n must be positive");
  hipStream_t s = static_cast<hipStream_t>(stream);
  adc_accumulate_kernel<<<grid_for(uint64_t(n), 256), 256, 0, s>>>(grad_mean, n, stat);
  FGS_LAUNCH_CHECK("adc_accumulate_kernel");
  return FGS_OK;
}

extern "C" int fgs_adc_densify(const fgs_gaussians *g, const fgs_gaussian_grads *m, const fgs_gaussian_grads *v,
                               const float *stat, const float *normals, const fgs_adc_params *p,
                               fgs_gaussians_out *g_out, fgs_gaussian_grads *m_out, fgs_gaussian_grads *v_out,
                               int64_t *n_out, fgs_workspace *ws, void *stream) {
  if (!g || !m || !v || !stat || !normals || !p || !g_out || !m_out || !v_out || !n_out || !ws)
    return fail(FGS_E_INVALID, "null argument");
  if (g->n <= 0 || !g->mean || !g->log_scale || !g->quat || !g->density) return fail(FGS_E_INVALID, "Gaussians");
  if (g->n > 0x7fffffff || p->n_max > 0x7fffffff) return fail(FGS_E_UNSUPPORTED, "more than 2^31 Gaussians");
  if (!(p->split_shrink > 0.f) || !(p->split_scale > 0.f) || !(p->prune_scale > 0.f))
    return fail(FGS_E_INVALID, "split_shrink, split_scale and prune_scale must be > 0");
  const uint64_t n = uint64_t(g->n);
  Carver c(nullptr);
  uint64_t o_cnt, o_code, o_key, o_val, o_key2, o_val2, o_scan, o_sort;
  c.take<unsigned long long>(2, &o_cnt);
  c.take<uint32_t>(n, &o_code);
  c.take<uint32_t>(n, &o_key);
  c.take<uint32_t>(n, &o_val);
  c.take<uint32_t>(n, &o_key2);
  c.take<uint32_t>(n, &o_val2);
  c.take<uint32_t>(n + 1, &o_scan);
  c.take<uint32_t>(std::max(scan_scratch_words(n), sort_scratch_words(n)), &o_sort);
  ws->needed = c.used;
  if (!ws->ptr || ws->bytes < ws->needed) return fail(FGS_E_CAPACITY, "workspace too small");
  ws->kind = 0;
  hipStream_t s = static_cast<hipStream_t>(stream);
  char *b = static_cast<char *>(ws->ptr);
  auto *counts = reinterpret_cast<unsigned long long *>(b + o_cnt);
  auto *code = reinterpret_cast<uint32_t *>(b + o_code);
  auto *key = reinterpret_cast<uint32_t *>(b + o_key);
  auto *val = reinterpret_cast<uint32_t *>(b + o_val);
  auto *cnt = reinterpret_cast<uint32_t *>(b + o_scan);
  auto *scratch = reinterpret_cast<uint32_t *>(b + o_sort);
  AdcThresholds th;
  th.grad = p->grad_threshold;
  th.ls_split = static_cast<float>(std::log(double(p->split_scale)));
  th.rho_prune = p->prune_density;
  th.ls_prune = static_cast<float>(std::log(double(p->prune_scale)));
  adc_zero_kernel<<<1, 64, 0, s>>>(counts);
  FGS_LAUNCH_CHECK("adc_zero_kernel");
  adc_classify_kernel<<<grid_for(n, 256), 256, 0, s>>>(*g, stat, th, code, key, val, counts);
  FGS_LAUNCH_CHECK("adc_classify_kernel");
  unsigned long long h[2];
  FGS_HIP(hipMemcpyAsync(h, counts, sizeof(h), hipMemcpyDeviceToHost, s));
  FGS_HIP(hipStreamSynchronize(s));
  const uint64_t n_surv = h[0], n_cand = h[1];
  if (p->n_max < 0 || n_surv > uint64_t(p->n_max))
    return fail(FGS_E_INVALID, "n_max is below the number of surviving Gaussians");
  const uint64_t room = uint64_t(p->n_max) - n_surv;
  if (n_cand > room) {
    uint32_t *sk, *sv;
    int st = radix_sort_pairs(key, val, reinterpret_cast<uint32_t *>(b + o_key2),
                              reinterpret_cast<uint32_t *>(b + o_val2), n, 32, scratch, &sk, &sv, s);
    if (st != FGS_OK) return st;
    adc_demote_kernel<<<grid_for(n_cand - room, 256), 256, 0, s>>>(sv, room, n_cand, code);
    FGS_LAUNCH_CHECK("adc_demote_kernel");
  }
  const uint64_t total = n_surv + std::min(n_cand, room);
  adc_count_kernel<<<grid_for(n, 256), 256, 0, s>>>(code, int64_t(n), cnt);
  FGS_LAUNCH_CHECK("adc_count_kernel");
  int st = exclusive_scan_u32(cnt, n, scratch, s);
  if (st != FGS_OK) return st;
  AdcOut o{*g_out, *m_out, *v_out, int64_t(total)};
  const float shrink = p->split_shrink;
  adc_emit_kernel<<<grid_for(n, 256), 256, 0, s>>>(*g, *m, *v, code, cnt, normals,
                                                   static_cast<float>(std::log(double(shrink))),
                                                   static_cast<float>(0.5 * double(shrink) * shrink * shrink), o);
  FGS_LAUNCH_CHECK("adc_emit_kernel");
  *n_out = int64_t(total);
  return FGS_OK;
}
