// C ABI of the learned-null threshold network and the greedy-step gate.
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstdio>
#include <algorithm>
#include <cstring>
#include <functional>
#include <vector>

#include "../../include/ksgcmi.h"
#include "mlp.h"
#include "runtime.h"

using namespace ksg;


#define KSG_HIP_RAW(expr)                    \
  do {                                       \
    if ((expr) != hipSuccess) {              \
      (void)hipGetLastError();               \
      return KSG_EDEVICE;                    \
    }                                        \
  } while (0)

static uint16_t host_bf16(float f) {
  uint32_t u;
  std::memcpy(&u, &f, 4);
  u += 0x7FFFu + ((u >> 16) & 1u);
  return (uint16_t)(u >> 16);
}

extern "C" int ksg_mlp_create(ksg_ctx* c, ksg_mlp** out, const float* init) {
  if (!c) return KSG_EINVAL;
  if (!out || !init) return c->fail(KSG_EINVAL, "ksg_mlp_create: null argument");
  *out = nullptr;
  for (int i = 0; i < kNParams; ++i)
    if (!std::isfinite(init[i])) return c->fail(KSG_ENONFINITE, "ksg_mlp_create: non-finite parameter %d", i);
  KSG_HIP(c, hipSetDevice(c->device));
  ksg_mlp* m = new ksg_mlp();
  m->device = c->device;
  const int nb_max = 4096;
  bool ok = hipMalloc(&m->master, sizeof(float) * kNParams) == hipSuccess &&
            hipMalloc(&m->wbf16, sizeof(uint16_t) * kNParams) == hipSuccess &&
            hipMalloc(&m->adam_m, sizeof(float) * kNParams) == hipSuccess &&
            hipMalloc(&m->adam_v, sizeof(float) * kNParams) == hipSuccess &&
            hipMalloc(&m->mu, sizeof(float) * kNIn) == hipSuccess &&
            hipMalloc(&m->sd, sizeof(float) * kNIn) == hipSuccess &&
            hipMalloc(&m->grad, sizeof(float) * kNParams) == hipSuccess &&
            hipMalloc(&m->loss, sizeof(float) * 2) == hipSuccess;
  if (!ok) {
    (void)hipGetLastError();
    ksg_mlp_destroy(m);
    return c->fail(KSG_ENOMEM, "ksg_mlp_create: allocation failed");
  }
  (void)nb_max;
  std::vector<uint16_t> wb(kNParams);
  for (int i = 0; i < kNParams; ++i) wb[i] = host_bf16(init[i]);
  for (int i = 0; i < kNIn; ++i) {
    m->h_mu[i] = 0.0f;
    m->h_sd[i] = 1.0f;
  }
  KSG_HIP(c, hipMemcpy(m->master, init, sizeof(float) * kNParams, hipMemcpyHostToDevice));
  KSG_HIP(c, hipMemcpy(m->wbf16, wb.data(), sizeof(uint16_t) * kNParams, hipMemcpyHostToDevice));
  KSG_HIP(c, hipMemset(m->adam_m, 0, sizeof(float) * kNParams));
  KSG_HIP(c, hipMemset(m->adam_v, 0, sizeof(float) * kNParams));
  KSG_HIP(c, hipMemcpy(m->mu, m->h_mu, sizeof(float) * kNIn, hipMemcpyHostToDevice));
  KSG_HIP(c, hipMemcpy(m->sd, m->h_sd, sizeof(float) * kNIn, hipMemcpyHostToDevice));
  *out = m;
  return KSG_OK;
}

extern "C" void ksg_mlp_destroy(ksg_mlp* m) {
  if (!m) return;
  (void)hipSetDevice(m->device);
  (void)hipDeviceSynchronize();
  for (void* p : {(void*)m->master, (void*)m->wbf16, (void*)m->adam_m, (void*)m->adam_v, (void*)m->mu,
                  (void*)m->sd, (void*)m->grad, (void*)m->loss, (void*)m->partials})
    if (p) (void)hipFree(p);
  (void)hipGetLastError();
  delete m;
}

extern "C" int ksg_mlp_set_norm(ksg_mlp* m, const float* mu, const float* sd) {
  if (!m || !mu || !sd) return KSG_EINVAL;
  for (int i = 0; i < kNIn; ++i)
    if (!std::isfinite(mu[i]) || !(sd[i] > 0.0f) || !std::isfinite(sd[i])) return KSG_EINVAL;
  KSG_HIP_RAW(hipSetDevice(m->device));
  std::memcpy(m->h_mu, mu, sizeof(float) * kNIn);
  std::memcpy(m->h_sd, sd, sizeof(float) * kNIn);
  KSG_HIP_RAW(hipMemcpy(m->mu, mu, sizeof(float) * kNIn, hipMemcpyHostToDevice));
  KSG_HIP_RAW(hipMemcpy(m->sd, sd, sizeof(float) * kNIn, hipMemcpyHostToDevice));
  return KSG_OK;
}

extern "C" int ksg_mlp_get_params(const ksg_mlp* m, float* out, int32_t bf16) {
  if (!m || !out) return KSG_EINVAL;
  KSG_HIP_RAW(hipSetDevice(m->device));
  KSG_HIP_RAW(hipDeviceSynchronize());
  if (bf16) {
    std::vector<uint16_t> wb(kNParams);
    KSG_HIP_RAW(hipMemcpy(wb.data(), m->wbf16, sizeof(uint16_t) * kNParams, hipMemcpyDeviceToHost));
    for (int i = 0; i < kNParams; ++i) {
      const uint32_t u = (uint32_t)wb[i] << 16;
      std::memcpy(&out[i], &u, 4);
    }
  } else {
    KSG_HIP_RAW(hipMemcpy(out, m->master, sizeof(float) * kNParams, hipMemcpyDeviceToHost));
  }
  return KSG_OK;
}

extern "C" int ksg_mlp_set_params(ksg_mlp* m, const float* params) {
  if (!m || !params) return KSG_EINVAL;
  for (int i = 0; i < kNParams; ++i)
    if (!std::isfinite(params[i])) return KSG_ENONFINITE;
  KSG_HIP_RAW(hipSetDevice(m->device));
  std::vector<uint16_t> wb(kNParams);
  for (int i = 0; i < kNParams; ++i) wb[i] = host_bf16(params[i]);
  KSG_HIP_RAW(hipDeviceSynchronize());
  KSG_HIP_RAW(hipMemcpy(m->master, params, sizeof(float) * kNParams, hipMemcpyHostToDevice));
  KSG_HIP_RAW(hipMemcpy(m->wbf16, wb.data(), sizeof(uint16_t) * kNParams, hipMemcpyHostToDevice));
  KSG_HIP_RAW(hipMemset(m->adam_m, 0, sizeof(float) * kNParams));
  KSG_HIP_RAW(hipMemset(m->adam_v, 0, sizeof(float) * kNParams));
  m->step = 0;
  return KSG_OK;
}

extern "C" int ksg_mlp_forward(ksg_ctx* c, const ksg_mlp* m, const float* feats, int64_t B, float* out) {
  if (!c) return KSG_EINVAL;
  if (!m || !feats || !out || B < 0) return c->fail(KSG_EINVAL, "ksg_mlp_forward: bad argument");
  if (m->device != c->device) return c->fail(KSG_EINVAL, "ksg_mlp_forward: network on another device");
  KSG_HIP(c, hipSetDevice(c->device));
  KSG_HIP(c, launch_mlp_forward(m->wbf16, m->mu, m->sd, feats, B, out, c->stream));
  return KSG_OK;
}

extern "C" int ksg_mlp_predict(ksg_ctx* c, const ksg_mlp* m, const float* feats, int64_t B, float* out) {
  return ksg_mlp_forward(c, m, feats, B, out);
}

static int ensure_partials(ksg_ctx* c, ksg_mlp* m, int64_t B) {
  const int nb = (int)((B + kGradRows - 1) / kGradRows);
  if (nb <= m->partial_blocks) return KSG_OK;
  KSG_HIP(c, hipStreamSynchronize(c->stream));
  if (m->partials) KSG_HIP(c, hipFree(m->partials));
  m->partials = nullptr;
  m->partial_blocks = 0;
  if (hipMalloc(&m->partials, sizeof(float) * (size_t)nb * (kNParams + 1)) != hipSuccess) {
    (void)hipGetLastError();
    m->partials = nullptr;
    return c->fail(KSG_ENOMEM, "gradient partials");
  }
  m->partial_blocks = nb;
  return KSG_OK;
}

extern "C" int ksg_mlp_grad(ksg_ctx* c, const ksg_mlp* mc, const float* feats, const float* targets,
                            int64_t B, float* grad, float* loss) {
  if (!c) return KSG_EINVAL;
  ksg_mlp* m = const_cast<ksg_mlp*>(mc);
  if (!m || !feats || !targets || !grad || !loss || B < 1 || B > (int64_t)1 << 30)
    return c->fail(KSG_EINVAL, "ksg_mlp_grad: bad argument");
  KSG_HIP(c, hipSetDevice(c->device));
  int st = ensure_partials(c, m, B);
  if (st) return st;
  KSG_HIP(c, launch_mlp_grad(m->wbf16, m->mu, m->sd, feats, targets, B, m->partials, grad, loss, nullptr,
                             c->stream));
  return KSG_OK;
}

extern "C" int ksg_mlp_train(ksg_ctx* c, ksg_mlp* m, const float* feats, const float* targets, int64_t B,
                             int32_t epochs, int32_t batch, float lr, float* loss_hist) {
  if (!c) return KSG_EINVAL;
  if (!m || !feats || !targets || B < 1 || epochs < 0 || batch < 1 || !(lr > 0.0f))
    return c->fail(KSG_EINVAL, "ksg_mlp_train: bad argument");
  KSG_HIP(c, hipSetDevice(c->device));
  int st = ensure_partials(c, m, std::min<int64_t>(batch, B));
  if (st) return st;
  const int64_t nbatch = (B + batch - 1) / batch;
  for (int e = 0; e < epochs; ++e) {
    KSG_HIP(c, hipMemsetAsync(m->loss + 1, 0, sizeof(float), c->stream));
    for (int64_t b0 = 0; b0 < B; b0 += batch) {
      const int64_t rows = std::min<int64_t>(batch, B - b0);
      KSG_HIP(c, launch_mlp_grad(m->wbf16, m->mu, m->sd, feats + b0 * kNIn, targets + b0 * kNOut, rows,
                                 m->partials, m->grad, m->loss, m->loss + 1, c->stream));
      m->step += 1;
      KSG_HIP(c, launch_adam(m->master, m->wbf16, m->grad, m->adam_m, m->adam_v, m->step, lr, c->stream));
    }
    if (loss_hist) {
      float acc = 0.0f;
      KSG_HIP(c, hipMemcpyAsync(&acc, m->loss + 1, sizeof(float), hipMemcpyDeviceToHost, c->stream));
      KSG_HIP(c, hipStreamSynchronize(c->stream));
      loss_hist[e] = acc / (float)nbatch;
    }
  }
  KSG_HIP(c, hipStreamSynchronize(c->stream));
  return KSG_OK;
}

static const char kMagic[8] = {'K', 'S', 'G', 'M', 'L', 'P', '1', 0};

extern "C" int ksg_mlp_save(const ksg_mlp* m, const char* path) {
  if (!m || !path) return KSG_EINVAL;
  std::vector<float> p(kNParams);
  int st = ksg_mlp_get_params(m, p.data(), 0);
  if (st) return st;
  FILE* f = std::fopen(path, "wb");
  if (!f) return KSG_EINVAL;
  const int32_t np = kNParams;
  bool ok = std::fwrite(kMagic, 1, 8, f) == 8 && std::fwrite(&np, 4, 1, f) == 1 &&
            std::fwrite(p.data(), 4, kNParams, f) == (size_t)kNParams &&
            std::fwrite(m->h_mu, 4, kNIn, f) == (size_t)kNIn && std::fwrite(m->h_sd, 4, kNIn, f) == (size_t)kNIn;
  ok = (std::fclose(f) == 0) && ok;
  return ok ? KSG_OK : KSG_EINVAL;
}

extern "C" int ksg_mlp_load(ksg_ctx* c, ksg_mlp** out, const char* path) {
  if (!c) return KSG_EINVAL;
  if (!out || !path) return c->fail(KSG_EINVAL, "ksg_mlp_load: null argument");
  FILE* f = std::fopen(path, "rb");
  if (!f) return c->fail(KSG_EINVAL, "ksg_mlp_load: cannot open %s", path);
  char magic[8];
  int32_t np = 0;
  std::vector<float> p(kNParams);
  float mu[kNIn], sd[kNIn];
  bool ok = std::fread(magic, 1, 8, f) == 8 && std::memcmp(magic, kMagic, 8) == 0 &&
            std::fread(&np, 4, 1, f) == 1 && np == kNParams &&
            std::fread(p.data(), 4, kNParams, f) == (size_t)kNParams && std::fread(mu, 4, kNIn, f) == (size_t)kNIn &&
            std::fread(sd, 4, kNIn, f) == (size_t)kNIn;
  std::fclose(f);
  if (!ok) return c->fail(KSG_EINVAL, "ksg_mlp_load: %s is not a threshold-network file", path);
  int st = ksg_mlp_create(c, out, p.data());
  if (st) return st;
  st = ksg_mlp_set_norm(*out, mu, sd);
  if (st) {
    ksg_mlp_destroy(*out);
    *out = nullptr;
    return c->fail(st, "ksg_mlp_load: bad feature normalisation");
  }
  return KSG_OK;
}

// ============================================================== features and gate

extern "C" int ksg_step_features(ksg_ctx* c, const double* orig_cmi, int32_t cands, const float* y,
                                 const float* cand, int64_t N, const int32_t* cand_idx, int32_t dx,
                                 int32_t dy, int32_t dz, int32_t k, int32_t n_perm, float* out) {
  if (!c) return KSG_EINVAL;
  if (!orig_cmi || !y || !cand || !cand_idx || !out || cands < 1 || N < 2 || N > INT32_MAX || n_perm < 1)
    return c->fail(KSG_EINVAL, "ksg_step_features: bad argument");
  int cmax = 0;
  for (int i = 0; i < cands; ++i) {
    if (cand_idx[i] < 0) return c->fail(KSG_EINVAL, "ksg_step_features: negative candidate index");
    cmax = std::max(cmax, cand_idx[i] + 1);
  }
  KSG_HIP(c, hipSetDevice(c->device));
  const size_t need = sizeof(double) * (size_t)(cmax + 1) * 3 + sizeof(int32_t) * cands + 64 * 4;
  int st = c->reserve(c->feat, need, "feature workspace");
  if (st) return st;
  double* mom = (double*)c->feat.ptr;
  double* ymom = mom + (size_t)cmax * 3;
  double* obs = ymom + 3;
  int32_t* idx = (int32_t*)(obs + 2);
  KSG_HIP(c, launch_column_moments(cand, N, cmax, (int)N, mom, c->stream));
  KSG_HIP(c, launch_column_moments(y, N, 1, (int)N, ymom, c->stream));
  KSG_HIP(c, hipMemcpyAsync(idx, cand_idx, sizeof(int32_t) * cands, hipMemcpyHostToDevice, c->stream));
  KSG_HIP(c, launch_step_features(orig_cmi, 1, cands, idx, ymom, mom, (int)N, dx, dy, dz, k, n_perm, out,
                                  obs, c->stream));
  KSG_HIP(c, hipStreamSynchronize(c->stream));
  return KSG_OK;
}

namespace ksg {

LearnedGate::~LearnedGate() {
  for (void* p : {(void*)mom, (void*)d_pool, (void*)d_feat, (void*)d_pred, (void*)d_obs, (void*)d_verdict})
    if (p) (void)hipFree(p);
  if (h) (void)hipHostFree(h);
  (void)hipGetLastError();
}

int LearnedGate::init(ksg_ctx* c, const ksg_mlp* net, const float* cand, int64_t n_pad, int nC,
                      const float* y, int nn) {
  m = net;
  C = nC;
  n = nn;
  if (m->device != c->device) return c->fail(KSG_EINVAL, "learned null lives on another device");
  bool ok = hipMalloc(&mom, sizeof(double) * (size_t)(C + 1) * 3) == hipSuccess &&
            hipMalloc(&d_pool, sizeof(int32_t) * C) == hipSuccess &&
            hipMalloc(&d_feat, sizeof(float) * kNIn) == hipSuccess &&
            hipMalloc(&d_pred, sizeof(float) * kNOut) == hipSuccess &&
            hipMalloc(&d_obs, sizeof(double) * 2) == hipSuccess &&
            hipMalloc(&d_verdict, sizeof(int)) == hipSuccess &&
            hipHostMalloc(&h, sizeof(Host), hipHostMallocDefault) == hipSuccess;
  if (!ok) {
    (void)hipGetLastError();
    return c->fail(KSG_ENOMEM, "learned gate workspace");
  }
  // The candidate columns and Y are fixed for the whole target: moments once.
  KSG_HIP(c, launch_column_moments(cand, n_pad, C, n, mom, c->stream));
  KSG_HIP(c, launch_column_moments(y, n_pad, 1, n, mom + (size_t)C * 3, c->stream));
  return KSG_OK;
}

int LearnedGate::decide(ksg_ctx* c, const double* d_cmi, int cands, int stride,
                        const std::vector<int>& pool, int dx, int dy, int dz, int k, int n_perm,
                        double margin_lo, double margin_hi, int* verdict, int* c_star, double* t_obs,
                        float* pred) {
  KSG_HIP(c, hipMemcpyAsync(d_pool, pool.data(), sizeof(int32_t) * cands, hipMemcpyHostToDevice, c->stream));
  KSG_HIP(c, launch_step_features(d_cmi, stride, cands, d_pool, mom + (size_t)C * 3, mom, n, dx, dy, dz, k,
                                  n_perm, d_feat, d_obs, c->stream));
  KSG_HIP(c, launch_mlp_forward(m->wbf16, m->mu, m->sd, d_feat, 1, d_pred, c->stream));
  KSG_HIP(c, launch_gate(d_pred, d_obs, n, margin_lo, margin_hi, d_verdict, c->stream));
  KSG_HIP(c, hipMemcpyAsync(&h->verdict, d_verdict, sizeof(int), hipMemcpyDeviceToHost, c->stream));
  KSG_HIP(c, hipMemcpyAsync(h->obs, d_obs, sizeof(double) * 2, hipMemcpyDeviceToHost, c->stream));
  KSG_HIP(c, hipMemcpyAsync(h->pred, d_pred, sizeof(float) * 2, hipMemcpyDeviceToHost, c->stream));
  KSG_HIP(c, hipStreamSynchronize(c->stream));
  pred[0] = h->pred[0];
  pred[1] = h->pred[1];
  *verdict = h->verdict;
  *t_obs = h->obs[0];
  *c_star = (int)h->obs[1];
  return KSG_OK;
}

}  // namespace ksg

// ============================================================== training data and calibration

extern "C" int ksg_null_examples(ksg_ctx* c, const double* table, int32_t rows, int32_t n_perm,
                                 const int32_t* row_cand, const int32_t* sub_off,
                                 const int32_t* sub_rows, int32_t n_sub, const float* cand, int32_t C,
                                 const float* y, int64_t N, int32_t dz, int32_t k, float* feats,
                                 float* targets, double* obs) {
  if (!c) return KSG_EINVAL;
  if (!table || !row_cand || !sub_off || !sub_rows || !cand || !y || !feats || !targets || !obs)
    return c->fail(KSG_EINVAL, "ksg_null_examples: null argument");
  if (rows < 1 || n_perm < 1 || n_perm > 4096 || n_sub < 1 || C < 1 || N < 2 || N > INT32_MAX || dz < 0 || k < 1)
    return c->fail(KSG_EINVAL, "ksg_null_examples: bad sizes");
  if (sub_off[0] != 0) return c->fail(KSG_EINVAL, "ksg_null_examples: sub_off[0] must be 0");
  for (int s = 0; s < n_sub; ++s)
    if (sub_off[s + 1] <= sub_off[s]) return c->fail(KSG_EINVAL, "ksg_null_examples: empty subset %d", s);
  const int nidx = sub_off[n_sub];
  for (int q = 0; q < nidx; ++q)
    if (sub_rows[q] < 0 || sub_rows[q] >= rows) return c->fail(KSG_EINVAL, "ksg_null_examples: row index out of range");
  for (int r = 0; r < rows; ++r)
    if (row_cand[r] < 0 || row_cand[r] >= C) return c->fail(KSG_EINVAL, "ksg_null_examples: candidate index out of range");
  KSG_HIP(c, hipSetDevice(c->device));
  const size_t b_mom = sizeof(double) * (size_t)(C + 1) * 3;
  const size_t b_idx = sizeof(int32_t) * ((size_t)n_sub + 1 + nidx + rows);
  int st = c->reserve(c->feat, b_mom + b_idx + 64, "example workspace");
  if (st) return st;
  double* mom = (double*)c->feat.ptr;
  int32_t* d_off = (int32_t*)((char*)c->feat.ptr + b_mom);
  int32_t* d_rows = d_off + n_sub + 1;
  int32_t* d_rc = d_rows + nidx;
  std::vector<int32_t> h(n_sub + 1 + nidx + rows);
  std::memcpy(h.data(), sub_off, sizeof(int32_t) * (n_sub + 1));
  std::memcpy(h.data() + n_sub + 1, sub_rows, sizeof(int32_t) * nidx);
  std::memcpy(h.data() + n_sub + 1 + nidx, row_cand, sizeof(int32_t) * rows);
  KSG_HIP(c, hipMemcpyAsync(d_off, h.data(), b_idx, hipMemcpyHostToDevice, c->stream));
  KSG_HIP(c, launch_column_moments(cand, N, C, (int)N, mom, c->stream));
  KSG_HIP(c, launch_column_moments(y, N, 1, (int)N, mom + (size_t)C * 3, c->stream));
  KSG_HIP(c, launch_null_examples(table, n_perm, d_off, d_rows, n_sub, d_rc, mom, mom + (size_t)C * 3,
                                  (int)N, 1, 1, dz, k, feats, targets, obs, c->stream));
  KSG_HIP(c, hipStreamSynchronize(c->stream));
  return KSG_OK;
}

extern "C" int ksg_mlp_fit_norm(ksg_ctx* c, ksg_mlp* m, const float* feats, int64_t B) {
  if (!c) return KSG_EINVAL;
  if (!m || !feats || B < 1) return c->fail(KSG_EINVAL, "ksg_mlp_fit_norm: bad argument");
  KSG_HIP(c, hipSetDevice(c->device));
  KSG_HIP(c, launch_feature_norm(feats, B, m->mu, m->sd, c->stream));
  KSG_HIP(c, hipMemcpyAsync(m->h_mu, m->mu, sizeof(float) * kNIn, hipMemcpyDeviceToHost, c->stream));
  KSG_HIP(c, hipMemcpyAsync(m->h_sd, m->sd, sizeof(float) * kNIn, hipMemcpyDeviceToHost, c->stream));
  KSG_HIP(c, hipStreamSynchronize(c->stream));
  return KSG_OK;
}

// Margins of the gate in units of s = |pred_0.01 - pred_0.05|: with u = (sqrt(N) t_obs -
// pred_0.05) / s, the gate includes when u > margin_hi and stops when u < -margin_lo.  Each
// margin is the smallest value >= 0 for which at most floor(rate/2 * B) examples are decided
// against their plain-test outcome on that side.
extern "C" int ksg_gate_calibrate_sides(ksg_ctx* c, const ksg_mlp* m, const float* feats, const double* obs,
                                        int64_t B, double rate_stop, double rate_include, double* margin_lo,
                                        double* margin_hi, double* fallback, int64_t* wrong) {
  if (!c) return KSG_EINVAL;
  if (!m || !feats || !obs || B < 1 || !(rate_stop >= 0 && rate_stop < 1) ||
      !(rate_include >= 0 && rate_include < 1) || !margin_lo || !margin_hi || !fallback || !wrong)
    return c->fail(KSG_EINVAL, "ksg_gate_calibrate: bad argument");
  KSG_HIP(c, hipSetDevice(c->device));
  int st = c->reserve(c->tmp, sizeof(float) * 2 * (size_t)B, "predictions");
  if (st) return st;
  KSG_HIP(c, launch_mlp_forward(m->wbf16, m->mu, m->sd, feats, B, (float*)c->tmp.ptr, c->stream));
  std::vector<float> pred(2 * (size_t)B);
  std::vector<double> ob(2 * (size_t)B);
  KSG_HIP(c, hipMemcpyAsync(pred.data(), c->tmp.ptr, sizeof(float) * 2 * B, hipMemcpyDeviceToHost, c->stream));
  KSG_HIP(c, hipMemcpyAsync(ob.data(), obs, sizeof(double) * 2 * B, hipMemcpyDeviceToHost, c->stream));
  KSG_HIP(c, hipStreamSynchronize(c->stream));
  std::vector<double> u_neg, u_pos;  // u of plainly non-significant / significant examples
  std::vector<double> u(B);
  for (int64_t i = 0; i < B; ++i) {
    const double s = std::max(std::fabs((double)pred[2 * i + 1] - (double)pred[2 * i]), 1e-30);
    u[i] = (ob[2 * i] - (double)pred[2 * i]) / s;
    (ob[2 * i + 1] > 0.5 ? u_pos : u_neg).push_back(u[i]);
  }
  const int64_t allow_hi = (int64_t)std::floor(rate_include * (double)B);
  const int64_t allow_lo = (int64_t)std::floor(rate_stop * (double)B);
  // margin_hi: at most `allow_hi` non-significant examples with u > margin_hi
  std::sort(u_neg.begin(), u_neg.end(), std::greater<double>());
  double hi = 0.0;
  if ((int64_t)u_neg.size() > allow_hi) hi = std::max(0.0, u_neg[allow_hi]);
  // margin_lo: at most `allow_lo` significant examples with u < -margin_lo
  std::sort(u_pos.begin(), u_pos.end());
  double lo = 0.0;
  if ((int64_t)u_pos.size() > allow_lo) lo = std::max(0.0, -u_pos[allow_lo]);
  int64_t band = 0, bad = 0;
  for (int64_t i = 0; i < B; ++i) {
    const bool sig = ob[2 * i + 1] > 0.5;
    if (u[i] > hi) bad += !sig;
    else if (u[i] < -lo) bad += sig;
    else ++band;
  }
  *margin_lo = lo;
  *margin_hi = hi;
  *fallback = (double)band / (double)B;
  *wrong = bad;
  return KSG_OK;
}

extern "C" int ksg_gate_calibrate(ksg_ctx* c, const ksg_mlp* m, const float* feats, const double* obs,
                                  int64_t B, double rate, double* margin_lo, double* margin_hi,
                                  double* fallback, int64_t* wrong) {
  if (!c) return KSG_EINVAL;
  if (!(rate >= 0 && rate < 1)) return c->fail(KSG_EINVAL, "ksg_gate_calibrate: bad argument");
  return ksg_gate_calibrate_sides(c, m, feats, obs, B, rate / 2.0, rate / 2.0, margin_lo, margin_hi, fallback,
                                  wrong);
}
