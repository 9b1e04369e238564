// Learned-null kernels: column moments, step features, the 16-64-64-2 threshold network
// (BF16 parameters, FP32 accumulation) forward and backward passes, Adam, and the gate.
//
// The network is tiny (5,378 parameters); its kernels are written for exact, deterministic
// reductions rather than matrix-core throughput: every gradient is a fixed-order sum over
// rows (inside a block) and then over blocks.
#include <hip/hip_runtime.h>
#include <math.h>

#include "mlp.h"

namespace ksg {

__device__ __forceinline__ float bf16_to_f32(uint16_t b) { return __uint_as_float((uint32_t)b << 16); }

// Round to nearest BF16, ties to even (finite inputs).
__device__ __forceinline__ uint16_t f32_to_bf16(float f) {
  uint32_t u = __float_as_uint(f);
  u += 0x7FFFu + ((u >> 16) & 1u);
  return (uint16_t)(u >> 16);
}

__device__ __forceinline__ void load_params(const uint16_t* __restrict__ w, float* W) {
  for (int i = threadIdx.x; i < kNParams; i += blockDim.x) W[i] = bf16_to_f32(w[i]);
}

// ------------------------------------------------------------------ forward

__global__ __launch_bounds__(256) void mlp_forward_kernel(const uint16_t* __restrict__ w,
                                                          const float* __restrict__ mu,
                                                          const float* __restrict__ sd,
                                                          const float* __restrict__ feats, int64_t B,
                                                          float* __restrict__ out) {
  __shared__ float W[kNParams];
  load_params(w, W);
  __syncthreads();
  const int64_t r = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (r >= B) return;
  float x[kNIn], h1[kNH], h2[kNH];
#pragma unroll
  for (int i = 0; i < kNIn; ++i) x[i] = (feats[r * kNIn + i] - mu[i]) / sd[i];
#pragma unroll 4
  for (int o = 0; o < kNH; ++o) {
    float a = W[kOffB1 + o];
#pragma unroll
    for (int i = 0; i < kNIn; ++i) a = fmaf(W[kOffW1 + o * kNIn + i], x[i], a);
    h1[o] = fmaxf(a, 0.0f);
  }
#pragma unroll 4
  for (int o = 0; o < kNH; ++o) {
    float a = W[kOffB2 + o];
#pragma unroll
    for (int i = 0; i < kNH; ++i) a = fmaf(W[kOffW2 + o * kNH + i], h1[i], a);
    h2[o] = fmaxf(a, 0.0f);
  }
#pragma unroll
  for (int o = 0; o < kNOut; ++o) {
    float a = W[kOffB3 + o];
#pragma unroll
    for (int i = 0; i < kNH; ++i) a = fmaf(W[kOffW3 + o * kNH + i], h2[i], a);
    out[r * kNOut + o] = a;
  }
}

hipError_t launch_mlp_forward(const uint16_t* w, const float* mu, const float* sd, const float* feats,
                              int64_t B, float* out, hipStream_t stream) {
  if (B <= 0) return hipSuccess;
  hipLaunchKernelGGL(mlp_forward_kernel, dim3((unsigned)((B + 255) / 256)), dim3(256), 0, stream, w,
                     mu, sd, feats, B, out);
  return hipGetLastError();
}

// ------------------------------------------------------------------ backward

// Block b handles rows [b*kGradRows, (b+1)*kGradRows).  Phase 1 (one thread per row): forward
// pass and back-propagated activation gradients into LDS.  Phase 2 (all threads): per-parameter
// sums over the block's rows in row order.  partials[b][p] (p < 5378) and partials[b][5378] = loss.
constexpr int kRowStride = kNIn + 4 * kNH + kNOut;  // x | h1 | h2 | g_a1 | g_a2 | g_out

__global__ __launch_bounds__(256) void mlp_grad_kernel(const uint16_t* __restrict__ w,
                                                       const float* __restrict__ mu,
                                                       const float* __restrict__ sd,
                                                       const float* __restrict__ feats,
                                                       const float* __restrict__ targets, int64_t B,
                                                       float* __restrict__ partials) {
  __shared__ float W[kNParams];
  __shared__ float R[kGradRows * kRowStride];
  __shared__ float s_loss[kGradRows];
  load_params(w, W);
  __syncthreads();
  const int64_t r0 = (int64_t)blockIdx.x * kGradRows;
  const float inv_b = 1.0f / (float)B;
  if (threadIdx.x < kGradRows) {
    float* row = R + threadIdx.x * kRowStride;
    float* x = row;
    float* h1 = x + kNIn;
    float* h2 = h1 + kNH;
    float* ga1 = h2 + kNH;
    float* ga2 = ga1 + kNH;
    float* gout = ga2 + kNH;
    const int64_t r = r0 + threadIdx.x;
    float loss = 0.0f;
    if (r < B) {
      for (int i = 0; i < kNIn; ++i) x[i] = (feats[r * kNIn + i] - mu[i]) / sd[i];
      for (int o = 0; o < kNH; ++o) {
        float a = W[kOffB1 + o];
        for (int i = 0; i < kNIn; ++i) a = fmaf(W[kOffW1 + o * kNIn + i], x[i], a);
        h1[o] = fmaxf(a, 0.0f);
      }
      for (int o = 0; o < kNH; ++o) {
        float a = W[kOffB2 + o];
        for (int i = 0; i < kNH; ++i) a = fmaf(W[kOffW2 + o * kNH + i], h1[i], a);
        h2[o] = fmaxf(a, 0.0f);
      }
      for (int o = 0; o < kNOut; ++o) {
        float a = W[kOffB3 + o];
        for (int i = 0; i < kNH; ++i) a = fmaf(W[kOffW3 + o * kNH + i], h2[i], a);
        const float diff = a - targets[r * kNOut + o];
        loss = fmaf(0.5f * diff, diff, loss);
        gout[o] = diff * inv_b;
      }
      for (int i = 0; i < kNH; ++i) {
        float g = 0.0f;
        for (int o = 0; o < kNOut; ++o) g = fmaf(gout[o], W[kOffW3 + o * kNH + i], g);
        ga2[i] = h2[i] > 0.0f ? g : 0.0f;
      }
      for (int i = 0; i < kNH; ++i) {
        float g = 0.0f;
        for (int o = 0; o < kNH; ++o) g = fmaf(ga2[o], W[kOffW2 + o * kNH + i], g);
        ga1[i] = h1[i] > 0.0f ? g : 0.0f;
      }
    } else {
      for (int i = 0; i < kRowStride; ++i) row[i] = 0.0f;
    }
    s_loss[threadIdx.x] = loss * inv_b;
  }
  __syncthreads();
  float* part = partials + (int64_t)blockIdx.x * (kNParams + 1);
  for (int p = threadIdx.x; p < kNParams; p += blockDim.x) {
    int a_off, b_off;  // activation-gradient slot and input slot (-1: bias)
    if (p < kOffB1) { a_off = kNIn + 2 * kNH + p / kNIn; b_off = p % kNIn; }
    else if (p < kOffW2) { a_off = kNIn + 2 * kNH + (p - kOffB1); b_off = -1; }
    else if (p < kOffB2) { const int q = p - kOffW2; a_off = kNIn + 3 * kNH + q / kNH; b_off = kNIn + q % kNH; }
    else if (p < kOffW3) { a_off = kNIn + 3 * kNH + (p - kOffB2); b_off = -1; }
    else if (p < kOffB3) { const int q = p - kOffW3; a_off = kNIn + 4 * kNH + q / kNH; b_off = kNIn + kNH + q % kNH; }
    else { a_off = kNIn + 4 * kNH + (p - kOffB3); b_off = -1; }
    float g = 0.0f;
    for (int rr = 0; rr < kGradRows; ++rr) {
      const float* row = R + rr * kRowStride;
      g = b_off < 0 ? g + row[a_off] : fmaf(row[a_off], row[b_off], g);
    }
    part[p] = g;
  }
  if (threadIdx.x == 0) {
    float l = 0.0f;
    for (int rr = 0; rr < kGradRows; ++rr) l += s_loss[rr];
    part[kNParams] = l;
  }
}

// grad[p] = sum over blocks (in order) of partials[b][p]; loss likewise, also added to loss_acc.
__global__ __launch_bounds__(256) void mlp_grad_reduce_kernel(const float* __restrict__ partials, int nb,
                                                              float* __restrict__ grad,
                                                              float* __restrict__ loss,
                                                              float* __restrict__ loss_acc) {
  const int p = blockIdx.x * blockDim.x + threadIdx.x;
  if (p > kNParams) return;
  float g = 0.0f;
  for (int b = 0; b < nb; ++b) g += partials[(int64_t)b * (kNParams + 1) + p];
  if (p < kNParams) grad[p] = g;
  else {
    *loss = g;
    if (loss_acc) *loss_acc += g;
  }
}

hipError_t launch_mlp_grad(const uint16_t* w, const float* mu, const float* sd, const float* feats,
                           const float* targets, int64_t B, float* partials, float* grad, float* loss,
                           float* loss_acc, hipStream_t stream) {
  if (B <= 0) return hipErrorInvalidValue;
  const int nb = (int)((B + kGradRows - 1) / kGradRows);
  hipLaunchKernelGGL(mlp_grad_kernel, dim3(nb), dim3(256), 0, stream, w, mu, sd, feats, targets, B,
                     partials);
  hipLaunchKernelGGL(mlp_grad_reduce_kernel, dim3((kNParams + 1 + 255) / 256), dim3(256), 0, stream,
                     partials, nb, grad, loss, loss_acc);
  return hipGetLastError();
}

// ------------------------------------------------------------------ Adam

__global__ __launch_bounds__(256) void adam_kernel(float* __restrict__ master, uint16_t* __restrict__ w,
                                                   const float* __restrict__ grad, float* __restrict__ m,
                                                   float* __restrict__ v, float lr, float bc1, float bc2) {
  const int p = blockIdx.x * blockDim.x + threadIdx.x;
  if (p >= kNParams) return;
  const float g = grad[p];
  const float mm = 0.9f * m[p] + 0.1f * g;
  const float vv = 0.999f * v[p] + 0.001f * g * g;
  m[p] = mm;
  v[p] = vv;
  const float upd = lr * (mm / bc1) / (sqrtf(vv / bc2) + 1e-8f);
  const float nm = master[p] - upd;
  master[p] = nm;
  w[p] = f32_to_bf16(nm);
}

hipError_t launch_adam(float* master, uint16_t* w, const float* grad, float* m, float* v, int step,
                       float lr, hipStream_t stream) {
  const float bc1 = (float)(1.0 - pow(0.9, (double)step));
  const float bc2 = (float)(1.0 - pow(0.999, (double)step));
  hipLaunchKernelGGL(adam_kernel, dim3((kNParams + 255) / 256), dim3(256), 0, stream, master, w, grad, m,
                     v, lr, bc1, bc2);
  return hipGetLastError();
}

__global__ void round_bf16_kernel(const float* __restrict__ master, uint16_t* __restrict__ w) {
  const int p = blockIdx.x * blockDim.x + threadIdx.x;
  if (p < kNParams) w[p] = f32_to_bf16(master[p]);
}

hipError_t launch_round_bf16(const float* master, uint16_t* w, hipStream_t stream) {
  hipLaunchKernelGGL(round_bf16_kernel, dim3((kNParams + 255) / 256), dim3(256), 0, stream, master, w);
  return hipGetLastError();
}

// ------------------------------------------------------------------ features

__device__ __forceinline__ double block_sum(double v, double* red) {
#pragma unroll
  for (int off = 32; off >= 1; off >>= 1) v += __shfl_xor(v, off, 64);
  const int wave = threadIdx.x >> 6;
  __syncthreads();
  if ((threadIdx.x & 63) == 0) red[wave] = v;
  __syncthreads();
  double s = 0.0;
  for (int i = 0; i < (int)(blockDim.x >> 6); ++i) s += red[i];
  return s;
}

// One block per column: population skewness, excess kurtosis and lag-1 autocorrelation,
// FP64 accumulation.  out[c][3].
__global__ __launch_bounds__(256) void column_moments_kernel(const float* __restrict__ base,
                                                             int64_t stride, int n,
                                                             double* __restrict__ out) {
  __shared__ double red[4];
  const float* col = base + (int64_t)blockIdx.x * stride;
  double s = 0.0;
  for (int i = threadIdx.x; i < n; i += blockDim.x) s += (double)col[i];
  const double mean = block_sum(s, red) / n;
  double m2 = 0, m3 = 0, m4 = 0, c1 = 0;
  for (int i = threadIdx.x; i < n; i += blockDim.x) {
    const double d = (double)col[i] - mean;
    const double d2 = d * d;
    m2 += d2;
    m3 += d2 * d;
    m4 += d2 * d2;
    if (i + 1 < n) c1 += d * ((double)col[i + 1] - mean);
  }
  m2 = block_sum(m2, red) / n;
  m3 = block_sum(m3, red) / n;
  m4 = block_sum(m4, red) / n;
  c1 = block_sum(c1, red) / n;
  if (threadIdx.x == 0) {
    double* o = out + (int64_t)blockIdx.x * 3;
    if (m2 > 0.0) {
      o[0] = m3 / (m2 * sqrt(m2));
      o[1] = m4 / (m2 * m2) - 3.0;
      o[2] = c1 / m2;
    } else {
      o[0] = o[1] = o[2] = 0.0;
    }
  }
}

hipError_t launch_column_moments(const float* base, int64_t stride, int n_cols, int n, double* out,
                                 hipStream_t stream) {
  if (n_cols <= 0) return hipSuccess;
  hipLaunchKernelGGL(column_moments_kernel, dim3(n_cols), dim3(256), 0, stream, base, stride, n, out);
  return hipGetLastError();
}

// Single thread: the 16 step features (see ksgcmi.h) from the c original CMIs (cmi[ci*stride]),
// the pooled candidates' moments and Y's moments.  obs = {t_obs, c_star}.
__global__ void step_features_kernel(const double* __restrict__ cmi, int stride, int c,
                                     const int32_t* __restrict__ pool, const double* __restrict__ y_mom,
                                     const double* __restrict__ cand_mom, int n, int dx, int dy,
                                     int dz, int k, int n_perm, float* __restrict__ feat,
                                     double* __restrict__ obs) {
  if (threadIdx.x != 0 || blockIdx.x != 0) return;
  int best = 0;
  double sum = 0.0;
  for (int i = 0; i < c; ++i) {
    const double v = cmi[(int64_t)i * stride];
    if (v > cmi[(int64_t)best * stride]) best = i;
    sum += v;
  }
  const double t_obs = cmi[(int64_t)best * stride];
  double second = t_obs;
  if (c > 1) {
    second = -INFINITY;
    for (int i = 0; i < c; ++i)
      if (i != best) second = fmax(second, cmi[(int64_t)i * stride]);
  }
  const double mean = sum / c;
  double var = 0.0;
  double sk = 0.0, ku = 0.0, ac = 0.0;
  for (int i = 0; i < c; ++i) {
    const double d = cmi[(int64_t)i * stride] - mean;
    var += d * d;
    const double* cm = cand_mom + (int64_t)pool[i] * 3;
    sk += cm[0];
    ku += cm[1];
    ac += fabs(cm[2]);
  }
  const double rn = sqrt((double)n);
  const double f[kNIn] = {log((double)n), (double)dx, (double)dy, (double)dz, (double)k,
                          log((double)c), log((double)n_perm), rn * t_obs, rn * second, rn * mean,
                          rn * sqrt(var / c), y_mom[0], y_mom[1], sk / c, ku / c, ac / c};
  for (int i = 0; i < kNIn; ++i) feat[i] = (float)f[i];
  obs[0] = t_obs;
  obs[1] = (double)best;
}

hipError_t launch_step_features(const double* cmi, int stride, int c, const int32_t* pool_idx,
                                const double* y_mom, const double* cand_mom, int n, int dx, int dy,
                                int dz, int k, int n_perm, float* feat, double* obs,
                                hipStream_t stream) {
  hipLaunchKernelGGL(step_features_kernel, dim3(1), dim3(64), 0, stream, cmi, stride, c, pool_idx,
                     y_mom, cand_mom, n, dx, dy, dz, k, n_perm, feat, obs);
  return hipGetLastError();
}

// One block per candidate subset of a step's surrogate table: the subset's max-statistic
// distribution gives one training example of the threshold network.  table: FP64 [rows][P+1]
// (column 0 = originals); the subset lists table rows; row_cand maps a row to its candidate
// column (for the moments).  Outputs: feats [n_sub][16] (the step features of the subset),
// targ [n_sub][2] = sqrt(N) * (tau_0.05, tau_0.01) (ceil(alpha P)-th largest per-round maximum),
// obs [n_sub][2] = (sqrt(N) * t_obs, 1 if the plain test is significant at 0.05 else 0).
constexpr int kMaxPermEx = 4096;

__global__ __launch_bounds__(256) void null_examples_kernel(
    const double* __restrict__ table, int P, const int32_t* __restrict__ sub_off,
    const int32_t* __restrict__ sub_rows, const int32_t* __restrict__ row_cand,
    const double* __restrict__ cand_mom, const double* __restrict__ y_mom, int n, int dx, int dy,
    int dz, int k, float* __restrict__ feats, float* __restrict__ targ, double* __restrict__ obs) {
  __shared__ double tmax[kMaxPermEx];
  __shared__ int s_count;
  const int sb = blockIdx.x;
  const int r0 = sub_off[sb], r1 = sub_off[sb + 1];
  const int c = r1 - r0;
  if (threadIdx.x == 0) s_count = 0;
  __syncthreads();
  // observed statistic and its candidate (lowest row position wins ties)
  double t_obs = table[(int64_t)sub_rows[r0] * (P + 1)];
  for (int q = r0 + 1; q < r1; ++q) t_obs = fmax(t_obs, table[(int64_t)sub_rows[q] * (P + 1)]);
  int local = 0;
  for (int p = threadIdx.x; p < P; p += blockDim.x) {
    double m = table[(int64_t)sub_rows[r0] * (P + 1) + p + 1];
    for (int q = r0 + 1; q < r1; ++q) m = fmax(m, table[(int64_t)sub_rows[q] * (P + 1) + p + 1]);
    tmax[p] = m;
    local += m >= t_obs ? 1 : 0;
  }
  atomicAdd(&s_count, local);
  __syncthreads();
  const int rk05 = min(max((int)ceil(0.05 * P), 1), P);
  const int rk01 = min(max((int)ceil(0.01 * P), 1), P);
  const double rn = sqrt((double)n);
  for (int p = threadIdx.x; p < P; p += blockDim.x) {
    const double v = tmax[p];
    int rank = 0;
    for (int q = 0; q < P; ++q) rank += (tmax[q] > v) || (tmax[q] == v && q < p);
    if (rank == rk05 - 1) targ[sb * 2 + 0] = (float)(rn * v);
    if (rank == rk01 - 1) targ[sb * 2 + 1] = (float)(rn * v);
  }
  if (threadIdx.x == 0) {
    double first = -INFINITY, second = -INFINITY, sum = 0.0;
    int best = -1;
    for (int q = r0; q < r1; ++q) {
      const double v = table[(int64_t)sub_rows[q] * (P + 1)];
      sum += v;
      if (best < 0 || v > first) {
        best = q;
        first = v;
      }
    }
    for (int q = r0; q < r1; ++q)
      if (q != best) second = fmax(second, table[(int64_t)sub_rows[q] * (P + 1)]);
    if (c == 1) second = first;
    const double mean = sum / c;
    double var = 0.0, sk = 0.0, ku = 0.0, ac = 0.0;
    for (int q = r0; q < r1; ++q) {
      const double d = table[(int64_t)sub_rows[q] * (P + 1)] - mean;
      var += d * d;
      const double* cm = cand_mom + (int64_t)row_cand[sub_rows[q]] * 3;
      sk += cm[0];
      ku += cm[1];
      ac += fabs(cm[2]);
    }
    const double f[kNIn] = {log((double)n), (double)dx, (double)dy, (double)dz, (double)k,
                            log((double)c), log((double)P), rn * first, rn * second, rn * mean,
                            rn * sqrt(var / c), y_mom[0], y_mom[1], sk / c, ku / c, ac / c};
    for (int i = 0; i < kNIn; ++i) feats[sb * kNIn + i] = (float)f[i];
    obs[sb * 2 + 0] = rn * t_obs;
    obs[sb * 2 + 1] = ((double)s_count / (double)P) < 0.05 ? 1.0 : 0.0;
  }
}

hipError_t launch_null_examples(const double* table, int P, const int32_t* sub_off,
                                const int32_t* sub_rows, int n_sub, const int32_t* row_cand,
                                const double* cand_mom, const double* y_mom, int n, int dx, int dy,
                                int dz, int k, float* feats, float* targ, double* obs,
                                hipStream_t stream) {
  if (n_sub <= 0) return hipSuccess;
  if (P < 1 || P > kMaxPermEx) return hipErrorInvalidValue;
  hipLaunchKernelGGL(null_examples_kernel, dim3(n_sub), dim3(256), 0, stream, table, P, sub_off,
                     sub_rows, row_cand, cand_mom, y_mom, n, dx, dy, dz, k, feats, targ, obs);
  return hipGetLastError();
}

// verdict: +1 include (t_obs clearly above the predicted 5% threshold), -1 stop (clearly
// below), 0 borderline (run the surrogates).  The network predicts sqrt(N) * tau, so the
// comparison is made on sqrt(N) * t_obs; s = |pred_0.01 - pred_0.05|.
__global__ void gate_kernel(const float* __restrict__ pred, const double* __restrict__ obs, int n,
                            double margin_lo, double margin_hi, int* __restrict__ verdict) {
  if (threadIdx.x != 0 || blockIdx.x != 0) return;
  const double t = sqrt((double)n) * obs[0];
  const double t05 = (double)pred[0];
  const double s = fabs((double)pred[1] - t05);
  *verdict = t > t05 + margin_hi * s ? 1 : (t < t05 - margin_lo * s ? -1 : 0);
}

// Per-feature mean and population standard deviation of feats [B][16] (FP64 accumulation, one
// block per feature, fixed-order reduction); sd falls back to 1 for a constant feature.
__global__ __launch_bounds__(256) void feature_norm_kernel(const float* __restrict__ feats, int64_t B,
                                                           float* __restrict__ mu, float* __restrict__ sd) {
  __shared__ double red[4];
  const int f = blockIdx.x;
  double s = 0.0;
  for (int64_t r = threadIdx.x; r < B; r += blockDim.x) s += (double)feats[r * kNIn + f];
  const double mean = block_sum(s, red) / (double)B;
  double v = 0.0;
  for (int64_t r = threadIdx.x; r < B; r += blockDim.x) {
    const double d = (double)feats[r * kNIn + f] - mean;
    v += d * d;
  }
  const double var = block_sum(v, red) / (double)B;
  if (threadIdx.x == 0) {
    mu[f] = (float)mean;
    const float sdv = (float)sqrt(var);
    sd[f] = sdv > 1e-12f ? sdv : 1.0f;
  }
}

hipError_t launch_feature_norm(const float* feats, int64_t B, float* mu, float* sd, hipStream_t stream) {
  hipLaunchKernelGGL(feature_norm_kernel, dim3(kNIn), dim3(256), 0, stream, feats, B, mu, sd);
  return hipGetLastError();
}

hipError_t launch_gate(const float* pred, const double* obs, int n, double margin_lo, double margin_hi,
                       int* verdict, hipStream_t stream) {
  hipLaunchKernelGGL(gate_kernel, dim3(1), dim3(64), 0, stream, pred, obs, n, margin_lo, margin_hi,
                     verdict);
  return hipGetLastError();
}

}  // namespace ksg
