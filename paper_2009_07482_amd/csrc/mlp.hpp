// Learned cost model: a 3-layer perceptron that predicts the natural log of an op's duration in
// microseconds from a feature vector of the op (kind, shape, bytes, dtype, streams in flight).
// It is trained on the GPU from runtime-recorded op times (forward, back-propagation and Adam
// kernels in mlp.hip) and evaluated by the EFT mapper in place of the roofline heuristic.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>
#include <memory>
#include <mutex>
#include <vector>

#include "core.hpp"

namespace psc {

constexpr int kMlpF = kFeatures;
constexpr int kMlpH = 64;   // hidden units per layer
// Flat parameter layout (float32): W1 (H x F, row-major), b1 (H), W2 (H x H), b2 (H), W3 (H), b3 (1).
constexpr int kMlpW1 = 0;
constexpr int kMlpB1 = kMlpW1 + kMlpH * kMlpF;
constexpr int kMlpW2 = kMlpB1 + kMlpH;
constexpr int kMlpB2 = kMlpW2 + kMlpH * kMlpH;
constexpr int kMlpW3 = kMlpB2 + kMlpH;
constexpr int kMlpB3 = kMlpW3 + kMlpH;
constexpr int kMlpP = kMlpB3 + 1;
// Largest sample count of the allocation-free gradient (its fixed scratch holds this many).
constexpr int64_t kMlpStaticMax = 4096;

struct MlpTrainOpts {
  int32_t epochs = 50;
  int32_t batch = 256;
  float lr = 1e-3f, beta1 = 0.9f, beta2 = 0.999f, eps = 1e-8f;
  uint64_t shuffle_seed = 0;  // 0: samples in their given order every epoch
};

// Everything training needs to resume: parameters, Adam moments and step count, feature scaling.
struct MlpState {
  std::vector<float> params, m, v;   // kMlpP each
  float mean[kMlpF], std_[kMlpF];
  int64_t step = 0;
};

}  // namespace psc

struct psc_mlp {
  int device = 0;
  hipStream_t stream = nullptr;
  float *params = nullptr, *m = nullptr, *v = nullptr;  // device, kMlpP each
  float *norm = nullptr;                                // device: mean[F], 1/std[F]
  float h_mean[psc::kMlpF], h_std[psc::kMlpF];
  int64_t step = 0;                                     // Adam steps taken
  // device scratch for a batch / a prediction set, grown on demand
  int64_t cap = 0;
  float *x = nullptr, *t = nullptr, *z1 = nullptr, *z2 = nullptr, *y = nullptr;
  float *dz1 = nullptr, *dz2 = nullptr, *dy = nullptr, *g = nullptr;
  int32_t *idx = nullptr;
  std::mutex mu;  // scratch use (predictions are requested through const handles)
  ~psc_mlp();
};

namespace psc {

psc_mlp *mlp_create(int device);
void mlp_set_params(psc_mlp &m, const float *p);
void mlp_get_params(psc_mlp &m, float *p);
void mlp_set_norm(psc_mlp &m, const float *mean, const float *std_);
void mlp_predict(psc_mlp &m, const float *x, int64_t n, float *y);
double mlp_grad(psc_mlp &m, const float *x, const float *t, int64_t n, float *grads);
double mlp_grad_static(psc_mlp &m, const float *x, const float *t, int64_t n, float *grads);
void mlp_get_state(psc_mlp &m, MlpState &st);
void mlp_put_state(psc_mlp &m, const MlpState &st);   // state already validated
void mlp_train(psc_mlp &m, const float *x, const float *t, int64_t n, const MlpTrainOpts &o, float *epoch_loss);


}  // namespace psc
