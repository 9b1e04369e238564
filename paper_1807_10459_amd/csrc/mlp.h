// Learned-null threshold network: device-side state and the greedy-step gate.
#pragma once

#include <hip/hip_runtime.h>

#include <vector>

#include "../../include/ksgcmi.h"
#include "internal.h"

struct ksg_ctx;

namespace ksg {

constexpr int kNIn = 16, kNH = 64, kNOut = 2;
constexpr int kNParams = kNH * kNIn + kNH + kNH * kNH + kNH + kNOut * kNH + kNOut;  // 5378
constexpr int kOffW1 = 0, kOffB1 = kOffW1 + kNH * kNIn, kOffW2 = kOffB1 + kNH,
              kOffB2 = kOffW2 + kNH * kNH, kOffW3 = kOffB2 + kNH, kOffB3 = kOffW3 + kNOut * kNH;
static_assert(kOffB3 + kNOut == kNParams, "parameter layout");
constexpr int kGradRows = 64;  // rows per gradient block

}  // namespace ksg

struct ksg_mlp {
  int device = 0;
  float* master = nullptr;    // FP32 master parameters [5378]
  uint16_t* wbf16 = nullptr;  // BF16 parameters in use [5378]
  float* adam_m = nullptr;
  float* adam_v = nullptr;
  float* mu = nullptr;  // feature standardisation [16]
  float* sd = nullptr;
  float h_mu[ksg::kNIn];
  float h_sd[ksg::kNIn];
  int step = 0;
  float* grad = nullptr;      // [5378]
  float* loss = nullptr;      // [2]: minibatch loss, epoch accumulator
  float* partials = nullptr;  // [blocks][5378 + 1]
  int partial_blocks = 0;
};

namespace ksg {

hipError_t launch_mlp_forward(const uint16_t* w, const float* mu, const float* sd,
                              const float* feats, int64_t B, float* out, hipStream_t stream);
hipError_t launch_mlp_grad(const uint16_t* w, const float* mu, const float* sd, const float* feats,
                           const float* targets, int64_t B, float* partials, float* grad,
                           float* loss, float* loss_acc, hipStream_t stream);
hipError_t launch_adam(float* master, uint16_t* w, const float* grad, float* m, float* v, int step,
                       float lr, hipStream_t stream);
hipError_t launch_round_bf16(const float* master, uint16_t* w, hipStream_t stream);
hipError_t launch_column_moments(const float* base, int64_t stride, int n_cols, int n,
                                 double* out, hipStream_t stream);
hipError_t launch_step_features(const double* cmi, int stride, int c, const int32_t* pool_idx,
                                const double* y_mom, const double* cand_mom, int n, int dx, int dy,
                                int dz, int k, int n_perm, float* feat, double* obs,
                                hipStream_t stream);
hipError_t launch_null_examples(const double* table, int P, const int32_t* sub_off,
                                const int32_t* sub_rows, int n_sub, const int32_t* row_cand,
                                const double* cand_mom, const double* y_mom, int n, int dx, int dy,
                                int dz, int k, float* feats, float* targ, double* obs,
                                hipStream_t stream);
hipError_t launch_feature_norm(const float* feats, int64_t B, float* mu, float* sd, hipStream_t stream);
hipError_t launch_gate(const float* pred, const double* obs, int n, double margin_lo,
                       double margin_hi, int* verdict, hipStream_t stream);

// Per-target gate state used by select_parents.
struct LearnedGate {
  const ksg_mlp* m = nullptr;
  double* mom = nullptr;  // [C+1][3]: candidate moments, then Y's
  int C = 0, n = 0;
  int32_t* d_pool = nullptr;  // [C]
  float* d_feat = nullptr;    // [16]
  float* d_pred = nullptr;    // [2]
  double* d_obs = nullptr;    // [2]: t_obs, c_star
  int* d_verdict = nullptr;
  struct Host {
    int verdict;
    int pad;
    double obs[2];
    float pred[2];
  }* h = nullptr;  // pinned
  ~LearnedGate();
  int init(ksg_ctx* c, const ksg_mlp* m, const float* cand, int64_t n_pad, int C, const float* y, int n);
  int decide(ksg_ctx* c, const double* d_cmi, int cands, int stride, const std::vector<int>& pool,
             int dx, int dy, int dz, int k, int n_perm, double margin_lo, double margin_hi,
             int* verdict, int* c_star, double* t_obs, float* pred);
};

}  // namespace ksg
