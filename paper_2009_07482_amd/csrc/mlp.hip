// Learned cost model on the GPU: forward pass, back-propagation and Adam for the 3-layer
// perceptron f -> 64 -> 64 -> 1 with ReLU (the paper names machine-learning assisted scheduling as future work, Sec. VII),
// trained on op times the runtime records.
//
// Training step on a batch of B samples (row indices into the uploaded sample set):
//   mlp_fwd     z1 = W1 xn + b1, h1 = relu(z1), z2 = W2 h1 + b2, h2 = relu(z2), y = W3 h2 + b3,
//               with xn the z-scored features; z1, z2 and y are kept per sample.
//   mlp_delta   dy = 2 (y - t) / B, dz2 = dy W3 * [z2 > 0], dz1 = (W2^T dz2) * [z1 > 0]
//   mlp_update  one thread per parameter sums its gradient over the batch in sample order
//               (deterministic), then applies Adam with bias-corrected moments.
// The network is ~9.9 kFLOP per sample forward, so every kernel is latency-bound: plain FP32
// vector FMAs with the weights staged in LDS, not matrix cores.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstring>
#include <numeric>
#include <random>
#include <string>

#include "mlp.hpp"

namespace psc {

#define MLP_HIP(call)                                                                          \
  do {                                                                                         \
    hipError_t e_ = (call);                                                                    \
    if (e_ != hipSuccess) fail(PSC_ERR_HIP, std::string(#call) + ": " + hipGetErrorString(e_)); \
  } while (0)

namespace {

constexpr int kSPB = 64;  // samples per block in mlp_fwd / mlp_delta (one per lane)
constexpr int kUPW = kMlpH / 4;  // hidden units per wave

// Block: 256 threads = 4 waves; lane l handles sample blockIdx.x * 64 + l, wave w handles hidden
// units [16w, 16w + 16).  Weight reads are wave-uniform (LDS broadcast).
__global__ __launch_bounds__(256) void mlp_fwd(const float *__restrict__ P, const float *__restrict__ norm,
                                               const float *__restrict__ X, const int32_t *__restrict__ idx,
                                               int32_t n, float *__restrict__ Z1, float *__restrict__ Z2,
                                               float *__restrict__ Y) {
  __shared__ float w[kMlpP];
  __shared__ float h1[kSPB][kMlpH + 1];
  __shared__ float red[4][kSPB];
  for (int i = threadIdx.x; i < kMlpP; i += 256) w[i] = P[i];
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  const int64_t s = int64_t(blockIdx.x) * kSPB + lane;
  const bool ok = s < n;
  float x[kMlpF];
  if (ok) {
    const int64_t r = idx ? idx[s] : s;
#pragma unroll
    for (int f = 0; f < kMlpF; ++f) x[f] = (X[r * kMlpF + f] - norm[f]) * norm[kMlpF + f];
  } else {
#pragma unroll
    for (int f = 0; f < kMlpF; ++f) x[f] = 0.0f;
  }
  __syncthreads();
#pragma unroll 4
  for (int u = 0; u < kUPW; ++u) {
    const int j = wv * kUPW + u;
    float z = w[kMlpB1 + j];
#pragma unroll
    for (int f = 0; f < kMlpF; ++f) z = fmaf(w[kMlpW1 + j * kMlpF + f], x[f], z);
    if (ok) Z1[s * kMlpH + j] = z;
    h1[lane][j] = fmaxf(z, 0.0f);
  }
  __syncthreads();
  float acc = 0.0f;
  for (int u = 0; u < kUPW; ++u) {
    const int j = wv * kUPW + u;
    float z = w[kMlpB2 + j];
#pragma unroll 16
    for (int i = 0; i < kMlpH; ++i) z = fmaf(w[kMlpW2 + j * kMlpH + i], h1[lane][i], z);
    if (ok) Z2[s * kMlpH + j] = z;
    acc = fmaf(w[kMlpW3 + j], fmaxf(z, 0.0f), acc);
  }
  red[wv][lane] = acc;
  __syncthreads();
  if (wv == 0 && ok) Y[s] = w[kMlpB3] + ((red[0][lane] + red[1][lane]) + (red[2][lane] + red[3][lane]));
}

// Same block layout as mlp_fwd.  scale = 2 / B (the derivative of the batch-mean squared error).
__global__ __launch_bounds__(256) void mlp_delta(const float *__restrict__ P, const float *__restrict__ T,
                                                 const int32_t *__restrict__ idx, int32_t n, float scale,
                                                 const float *__restrict__ Z1, const float *__restrict__ Z2,
                                                 const float *__restrict__ Y, float *__restrict__ DZ1,
                                                 float *__restrict__ DZ2, float *__restrict__ DY) {
  __shared__ float w2[kMlpH * kMlpH];
  __shared__ float w3[kMlpH];
  __shared__ float d2[kSPB][kMlpH + 1];
  for (int i = threadIdx.x; i < kMlpH * kMlpH; i += 256) w2[i] = P[kMlpW2 + i];
  if (threadIdx.x < kMlpH) w3[threadIdx.x] = P[kMlpW3 + threadIdx.x];
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  const int64_t s = int64_t(blockIdx.x) * kSPB + lane;
  const bool ok = s < n;
  const float dy = ok ? scale * (Y[s] - T[idx ? idx[s] : s]) : 0.0f;
  __syncthreads();
  for (int u = 0; u < kUPW; ++u) {
    const int j = wv * kUPW + u;
    const float d = ok && Z2[s * kMlpH + j] > 0.0f ? dy * w3[j] : 0.0f;
    if (ok) DZ2[s * kMlpH + j] = d;
    d2[lane][j] = d;
  }
  __syncthreads();
  for (int u = 0; u < kUPW; ++u) {
    const int i = wv * kUPW + u;
    float acc = 0.0f;
#pragma unroll 16
    for (int j = 0; j < kMlpH; ++j) acc = fmaf(w2[j * kMlpH + i], d2[lane][j], acc);
    if (ok) DZ1[s * kMlpH + i] = Z1[s * kMlpH + i] > 0.0f ? acc : 0.0f;
  }
  if (wv == 0 && ok) DY[s] = dy;
}

struct UpdateArgs {
  float *P, *M, *V, *G;  // G may be null
  const float *norm, *X;
  const int32_t *idx;
  const float *Z1, *Z2, *DZ1, *DZ2, *DY;
  int32_t n;
  int32_t update;        // apply Adam
  float lr, beta1, beta2, eps, c1, c2;  // c1 = 1 / (1 - beta1^t), c2 = 1 / (1 - beta2^t)
};

// One thread per parameter; the batch sum runs in sample order.
__global__ __launch_bounds__(256) void mlp_update(UpdateArgs a) {
  const int p = blockIdx.x * 256 + threadIdx.x;
  if (p >= kMlpP) return;
  float g = 0.0f;
  if (p < kMlpB1) {
    const int i = p / kMlpF, f = p % kMlpF;
    const float mu = a.norm[f], is = a.norm[kMlpF + f];
    for (int32_t s = 0; s < a.n; ++s) {
      const int64_t r = a.idx ? a.idx[s] : s;
      g = fmaf(a.DZ1[int64_t(s) * kMlpH + i], (a.X[r * kMlpF + f] - mu) * is, g);
    }
  } else if (p < kMlpW2) {
    const int i = p - kMlpB1;
    for (int32_t s = 0; s < a.n; ++s) g += a.DZ1[int64_t(s) * kMlpH + i];
  } else if (p < kMlpB2) {
    const int i = (p - kMlpW2) / kMlpH, j = (p - kMlpW2) % kMlpH;
    for (int32_t s = 0; s < a.n; ++s)
      g = fmaf(a.DZ2[int64_t(s) * kMlpH + i], fmaxf(a.Z1[int64_t(s) * kMlpH + j], 0.0f), g);
  } else if (p < kMlpW3) {
    const int i = p - kMlpB2;
    for (int32_t s = 0; s < a.n; ++s) g += a.DZ2[int64_t(s) * kMlpH + i];
  } else if (p < kMlpB3) {
    const int j = p - kMlpW3;
    for (int32_t s = 0; s < a.n; ++s) g = fmaf(a.DY[s], fmaxf(a.Z2[int64_t(s) * kMlpH + j], 0.0f), g);
  } else {
    for (int32_t s = 0; s < a.n; ++s) g += a.DY[s];
  }
  if (a.G) a.G[p] = g;
  if (a.update) {
    const float m = a.beta1 * a.M[p] + (1.0f - a.beta1) * g;
    const float v = a.beta2 * a.V[p] + (1.0f - a.beta2) * g * g;
    a.M[p] = m;
    a.V[p] = v;
    a.P[p] -= a.lr * (m * a.c1) / (sqrtf(v * a.c2) + a.eps);
  }
}

void ensure_cap(psc_mlp &m, int64_t n) {
  if (n <= m.cap) return;
  const int64_t c = std::max<int64_t>(n, 2 * m.cap);
  float **fl[] = {&m.x, &m.t, &m.z1, &m.z2, &m.y, &m.dz1, &m.dz2, &m.dy};
  for (float **p : fl)
    if (*p) { MLP_HIP(hipFree(*p)); *p = nullptr; }
  if (m.idx) { MLP_HIP(hipFree(m.idx)); m.idx = nullptr; }
  m.cap = 0;
  MLP_HIP(hipMalloc(&m.x, size_t(c) * kMlpF * 4));
  MLP_HIP(hipMalloc(&m.t, size_t(c) * 4));
  MLP_HIP(hipMalloc(&m.z1, size_t(c) * kMlpH * 4));
  MLP_HIP(hipMalloc(&m.z2, size_t(c) * kMlpH * 4));
  MLP_HIP(hipMalloc(&m.y, size_t(c) * 4));
  MLP_HIP(hipMalloc(&m.dz1, size_t(c) * kMlpH * 4));
  MLP_HIP(hipMalloc(&m.dz2, size_t(c) * kMlpH * 4));
  MLP_HIP(hipMalloc(&m.dy, size_t(c) * 4));
  MLP_HIP(hipMalloc(&m.idx, size_t(c) * 4));
  m.cap = c;
}

unsigned blocks_for(int64_t n) { return unsigned((n + kSPB - 1) / kSPB); }

void check_n(int64_t n) {
  if (n < 1 || n > (int64_t(1) << 30)) fail(PSC_ERR_ARG, "sample count must be in [1, 2^30]");
}

// Device memory of one forward / backward pass: the samples (x, t), the per-sample activations
// (z1, z2, y) and the back-propagated errors (dz1, dz2, dy).  The model's own buffers (grown on
// demand) or the fixed scratch array of the allocation-free entry point.
struct Work {
  const float *x, *t;
  float *z1, *z2, *y, *dz1, *dz2, *dy;
};

Work work_of(psc_mlp &m) { return Work{m.x, m.t, m.z1, m.z2, m.y, m.dz1, m.dz2, m.dy}; }

// fwd over the first n uploaded samples (rows idx[0..n) if idx, else 0..n)
void launch_fwd(psc_mlp &m, const Work &w, const int32_t *idx, int64_t n) {
  const float *P = m.params, *norm = m.norm, *X = w.x;
  int32_t nn = int32_t(n);
  float *Z1 = w.z1, *Z2 = w.z2, *Y = w.y;
  void *args[] = {&P, &norm, &X, &idx, &nn, &Z1, &Z2, &Y};
  MLP_HIP(hipLaunchKernel(reinterpret_cast<const void *>(&mlp_fwd), dim3(blocks_for(n)), dim3(256), args, 0, m.stream));
}

void launch_fwd(psc_mlp &m, const int32_t *idx, int64_t n) { launch_fwd(m, work_of(m), idx, n); }

void launch_step(psc_mlp &m, const Work &w, const int32_t *idx, int64_t n, bool update, const MlpTrainOpts &o,
                 float *G) {
  launch_fwd(m, w, idx, n);
  {
    const float *P = m.params, *T = w.t, *Z1 = w.z1, *Z2 = w.z2, *Y = w.y;
    int32_t nn = int32_t(n);
    float scale = float(2.0 / double(n));
    float *DZ1 = w.dz1, *DZ2 = w.dz2, *DY = w.dy;
    void *args[] = {&P, &T, &idx, &nn, &scale, &Z1, &Z2, &Y, &DZ1, &DZ2, &DY};
    MLP_HIP(hipLaunchKernel(reinterpret_cast<const void *>(&mlp_delta), dim3(blocks_for(n)), dim3(256), args, 0,
                            m.stream));
  }
  UpdateArgs a{};
  a.P = m.params;
  a.M = m.m;
  a.V = m.v;
  a.G = G;
  a.norm = m.norm;
  a.X = w.x;
  a.idx = idx;
  a.Z1 = w.z1;
  a.Z2 = w.z2;
  a.DZ1 = w.dz1;
  a.DZ2 = w.dz2;
  a.DY = w.dy;
  a.n = int32_t(n);
  a.update = update ? 1 : 0;
  if (update) {
    ++m.step;
    a.lr = o.lr;
    a.beta1 = o.beta1;
    a.beta2 = o.beta2;
    a.eps = o.eps;
    a.c1 = float(1.0 / (1.0 - std::pow(double(o.beta1), double(m.step))));
    a.c2 = float(1.0 / (1.0 - std::pow(double(o.beta2), double(m.step))));
  }
  void *uargs[] = {&a};
  MLP_HIP(hipLaunchKernel(reinterpret_cast<const void *>(&mlp_update), dim3((kMlpP + 255) / 256), dim3(256), uargs, 0,
                          m.stream));
}

void launch_step(psc_mlp &m, const int32_t *idx, int64_t n, bool update, const MlpTrainOpts &o, float *G) {
  launch_step(m, work_of(m), idx, n, update, o, G);
}

double mse_of(const std::vector<float> &y, const float *t, int64_t n) {
  double acc = 0;
  for (int64_t i = 0; i < n; ++i) {
    const double d = double(y[i]) - double(t[i]);
    acc += d * d;
  }
  return acc / double(n);
}

void upload_x(psc_mlp &m, const float *x, int64_t n) {
  MLP_HIP(hipMemcpyAsync(m.x, x, size_t(n) * kMlpF * 4, hipMemcpyHostToDevice, m.stream));
}

}  // namespace

psc_mlp *mlp_create(int device) {
  int nd = 0;
  MLP_HIP(hipGetDeviceCount(&nd));
  if (device < 0 || device >= nd) fail(PSC_ERR_ARG, "device ordinal out of range");
  MLP_HIP(hipSetDevice(device));
  auto m = std::make_unique<psc_mlp>();
  m->device = device;
  MLP_HIP(hipStreamCreateWithFlags(&m->stream, hipStreamNonBlocking));
  MLP_HIP(hipMalloc(&m->params, kMlpP * 4));
  MLP_HIP(hipMalloc(&m->m, kMlpP * 4));
  MLP_HIP(hipMalloc(&m->v, kMlpP * 4));
  MLP_HIP(hipMalloc(&m->g, kMlpP * 4));
  MLP_HIP(hipMalloc(&m->norm, 2 * kMlpF * 4));
  std::vector<float> z(kMlpP, 0.0f);
  MLP_HIP(hipMemcpy(m->params, z.data(), kMlpP * 4, hipMemcpyHostToDevice));
  MLP_HIP(hipMemcpy(m->m, z.data(), kMlpP * 4, hipMemcpyHostToDevice));
  MLP_HIP(hipMemcpy(m->v, z.data(), kMlpP * 4, hipMemcpyHostToDevice));
  const float mean[kMlpF] = {}, sd[kMlpF] = {1, 1, 1, 1, 1, 1, 1, 1, 1, 1, 1, 1};
  mlp_set_norm(*m, mean, sd);
  return m.release();
}

void mlp_set_params(psc_mlp &m, const float *p) {
  std::lock_guard<std::mutex> lk(m.mu);
  MLP_HIP(hipSetDevice(m.device));
  std::vector<float> z(kMlpP, 0.0f);
  MLP_HIP(hipMemcpy(m.params, p, kMlpP * 4, hipMemcpyHostToDevice));
  MLP_HIP(hipMemcpy(m.m, z.data(), kMlpP * 4, hipMemcpyHostToDevice));
  MLP_HIP(hipMemcpy(m.v, z.data(), kMlpP * 4, hipMemcpyHostToDevice));
  m.step = 0;
}

void mlp_get_params(psc_mlp &m, float *p) {
  std::lock_guard<std::mutex> lk(m.mu);
  MLP_HIP(hipSetDevice(m.device));
  MLP_HIP(hipStreamSynchronize(m.stream));
  MLP_HIP(hipMemcpy(p, m.params, kMlpP * 4, hipMemcpyDeviceToHost));
}

void mlp_set_norm(psc_mlp &m, const float *mean, const float *std_) {
  float h[2 * kMlpF];
  for (int f = 0; f < kMlpF; ++f) {
    if (!(std_[f] > 0.0f) || !std::isfinite(std_[f]) || !std::isfinite(mean[f]))
      fail(PSC_ERR_ARG, "feature scales must be finite and positive");
    h[f] = mean[f];
    h[kMlpF + f] = 1.0f / std_[f];
    m.h_mean[f] = mean[f];
    m.h_std[f] = std_[f];
  }
  MLP_HIP(hipSetDevice(m.device));
  MLP_HIP(hipMemcpy(m.norm, h, sizeof(h), hipMemcpyHostToDevice));
}

void mlp_predict(psc_mlp &m, const float *x, int64_t n, float *y) {
  check_n(n);
  std::lock_guard<std::mutex> lk(m.mu);
  MLP_HIP(hipSetDevice(m.device));
  ensure_cap(m, n);
  upload_x(m, x, n);
  launch_fwd(m, nullptr, n);
  MLP_HIP(hipMemcpyAsync(y, m.y, size_t(n) * 4, hipMemcpyDeviceToHost, m.stream));
  MLP_HIP(hipStreamSynchronize(m.stream));
}

double mlp_grad(psc_mlp &m, const float *x, const float *t, int64_t n, float *grads) {
  check_n(n);
  std::lock_guard<std::mutex> lk(m.mu);
  MLP_HIP(hipSetDevice(m.device));
  ensure_cap(m, n);
  upload_x(m, x, n);
  MLP_HIP(hipMemcpyAsync(m.t, t, size_t(n) * 4, hipMemcpyHostToDevice, m.stream));
  launch_step(m, nullptr, n, false, MlpTrainOpts{}, m.g);
  std::vector<float> y(n);
  MLP_HIP(hipMemcpyAsync(y.data(), m.y, size_t(n) * 4, hipMemcpyDeviceToHost, m.stream));
  if (grads) MLP_HIP(hipMemcpyAsync(grads, m.g, kMlpP * 4, hipMemcpyDeviceToHost, m.stream));
  MLP_HIP(hipStreamSynchronize(m.stream));
  return mse_of(y, t, n);
}

// ---------------------------------------------------------------------------------------------
// Allocation-free gradient (psc_mlp_grad_static): the same kernels as mlp_grad, with every
// buffer of the pass in one fixed device array instead of memory the model allocates.
// ---------------------------------------------------------------------------------------------

namespace {

// Layout of the scratch array, in floats: x (max x F), t, z1, z2, y, dz1, dz2, dy, the gradient
// (kMlpP, padded) and the loss (one double).
constexpr int64_t kSMax = kMlpStaticMax;
constexpr int64_t kOffX = 0;
constexpr int64_t kOffT = kOffX + kSMax * kMlpF;
constexpr int64_t kOffZ1 = kOffT + kSMax;
constexpr int64_t kOffZ2 = kOffZ1 + kSMax * kMlpH;
constexpr int64_t kOffY = kOffZ2 + kSMax * kMlpH;
constexpr int64_t kOffDZ1 = kOffY + kSMax;
constexpr int64_t kOffDZ2 = kOffDZ1 + kSMax * kMlpH;
constexpr int64_t kOffDY = kOffDZ2 + kSMax * kMlpH;
constexpr int64_t kOffG = kOffDY + kSMax;
constexpr int64_t kOffLoss = kOffG + ((kMlpP + 63) / 64) * 64;
constexpr int64_t kScratchFloats = kOffLoss + 64;

// One copy per GPU, held until the process ends.  Host code never passes this name to a kernel or
// a copy: it is the host-side stand-in, and the device address comes from hipGetSymbolAddress.
static __device__ __align__(256) float scratch[kScratchFloats];

constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu[kMaxDevices];   // one call at a time per GPU: every call shares its array
float *g_scratch_ptr[kMaxDevices] = {};

float *scratch_of(int device) {
  if (g_scratch_ptr[device]) return g_scratch_ptr[device];
  void *p = nullptr;
  const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
  if (e != hipSuccess || p == nullptr)
    fail(PSC_ERR_HIP, std::string("hipGetSymbolAddress(scratch): ") + hipGetErrorString(e));
  g_scratch_ptr[device] = static_cast<float *>(p);
  return g_scratch_ptr[device];
}

// Mean squared error of y against t over n samples in float64: 256 threads, thread i sums samples
// i, i + 256, ... in order, then a fixed-order tree over the threads.
__global__ __launch_bounds__(256) void mlp_mse(const float *__restrict__ Y, const float *__restrict__ T, int32_t n,
                                               double *__restrict__ out) {
  __shared__ double part[256];
  double acc = 0.0;
  for (int32_t s = threadIdx.x; s < n; s += 256) {
    const double d = double(Y[s]) - double(T[s]);
    acc = fma(d, d, acc);
  }
  part[threadIdx.x] = acc;
  __syncthreads();
  for (int w = 128; w > 0; w >>= 1) {
    if (int(threadIdx.x) < w) part[threadIdx.x] += part[threadIdx.x + w];
    __syncthreads();
  }
  if (threadIdx.x == 0) out[0] = part[0] / double(n);
}

}  // namespace

double mlp_grad_static(psc_mlp &m, const float *x, const float *t, int64_t n, float *grads) {
  if (n < 1 || n > kMlpStaticMax)
    fail(PSC_ERR_ARG, "sample count must be in [1, " + std::to_string(kMlpStaticMax) + "] (the fixed scratch size)");
  if (m.device < 0 || m.device >= kMaxDevices) fail(PSC_ERR_ARG, "device ordinal out of range");
  std::lock_guard<std::mutex> lk(m.mu);
  std::lock_guard<std::mutex> sk(g_scratch_mu[m.device]);
  MLP_HIP(hipSetDevice(m.device));
  float *base = scratch_of(m.device);
  float *xs = base + kOffX, *ts = base + kOffT;
  const Work w{xs, ts, base + kOffZ1, base + kOffZ2, base + kOffY, base + kOffDZ1, base + kOffDZ2, base + kOffDY};
  float *G = base + kOffG;
  double *L = reinterpret_cast<double *>(base + kOffLoss);
  MLP_HIP(hipMemcpyAsync(xs, x, size_t(n) * kMlpF * 4, hipMemcpyHostToDevice, m.stream));
  MLP_HIP(hipMemcpyAsync(ts, t, size_t(n) * 4, hipMemcpyHostToDevice, m.stream));
  // every element the kernels read is written first in this call (x, t above; z, y, deltas by
  // the passes; G and the loss entirely), so nothing left by an earlier call is seen
  launch_step(m, w, nullptr, n, false, MlpTrainOpts{}, G);
  {
    const float *Y = w.y, *T = ts;
    int32_t nn = int32_t(n);
    void *args[] = {&Y, &T, &nn, &L};
    MLP_HIP(hipLaunchKernel(reinterpret_cast<const void *>(&mlp_mse), dim3(1), dim3(256), args, 0, m.stream));
  }
  double loss = 0.0;
  MLP_HIP(hipMemcpyAsync(&loss, L, sizeof(double), hipMemcpyDeviceToHost, m.stream));
  if (grads) MLP_HIP(hipMemcpyAsync(grads, G, kMlpP * 4, hipMemcpyDeviceToHost, m.stream));
  MLP_HIP(hipStreamSynchronize(m.stream));
  return loss;
}

void mlp_train(psc_mlp &m, const float *x, const float *t, int64_t n, const MlpTrainOpts &o, float *epoch_loss) {
  check_n(n);
  if (o.epochs < 1 || o.batch < 1) fail(PSC_ERR_ARG, "epochs and batch must be >= 1");
  if (!(o.lr > 0.0f) || !(o.beta1 >= 0.0f && o.beta1 < 1.0f) || !(o.beta2 >= 0.0f && o.beta2 < 1.0f) ||
      !(o.eps > 0.0f))
    fail(PSC_ERR_ARG, "Adam hyper-parameters out of range");
  std::lock_guard<std::mutex> lk(m.mu);
  MLP_HIP(hipSetDevice(m.device));
  ensure_cap(m, n);
  upload_x(m, x, n);
  MLP_HIP(hipMemcpyAsync(m.t, t, size_t(n) * 4, hipMemcpyHostToDevice, m.stream));
  std::vector<int32_t> order(n);
  std::iota(order.begin(), order.end(), 0);
  std::mt19937_64 gen(o.shuffle_seed);
  std::vector<float> y(n);
  for (int32_t e = 0; e < o.epochs; ++e) {
    if (o.shuffle_seed) std::shuffle(order.begin(), order.end(), gen);
    // the previous epoch's steps must be done with idx before it is overwritten
    MLP_HIP(hipStreamSynchronize(m.stream));
    MLP_HIP(hipMemcpyAsync(m.idx, order.data(), size_t(n) * 4, hipMemcpyHostToDevice, m.stream));
    for (int64_t b0 = 0; b0 < n; b0 += o.batch)
      launch_step(m, m.idx + b0, std::min<int64_t>(o.batch, n - b0), true, o, nullptr);
    if (epoch_loss) {
      launch_fwd(m, nullptr, n);
      MLP_HIP(hipMemcpyAsync(y.data(), m.y, size_t(n) * 4, hipMemcpyDeviceToHost, m.stream));
      MLP_HIP(hipStreamSynchronize(m.stream));
      epoch_loss[e] = float(mse_of(y, t, n));
    }
  }
  MLP_HIP(hipStreamSynchronize(m.stream));
}

void mlp_get_state(psc_mlp &m, MlpState &st) {
  std::lock_guard<std::mutex> lk(m.mu);
  MLP_HIP(hipSetDevice(m.device));
  MLP_HIP(hipStreamSynchronize(m.stream));
  st.params.resize(kMlpP);
  st.m.resize(kMlpP);
  st.v.resize(kMlpP);
  MLP_HIP(hipMemcpy(st.params.data(), m.params, kMlpP * 4, hipMemcpyDeviceToHost));
  MLP_HIP(hipMemcpy(st.m.data(), m.m, kMlpP * 4, hipMemcpyDeviceToHost));
  MLP_HIP(hipMemcpy(st.v.data(), m.v, kMlpP * 4, hipMemcpyDeviceToHost));
  std::copy(m.h_mean, m.h_mean + kMlpF, st.mean);
  std::copy(m.h_std, m.h_std + kMlpF, st.std_);
  st.step = m.step;
}

void mlp_put_state(psc_mlp &m, const MlpState &st) {
  mlp_set_norm(m, st.mean, st.std_);
  std::lock_guard<std::mutex> lk(m.mu);
  MLP_HIP(hipSetDevice(m.device));
  MLP_HIP(hipStreamSynchronize(m.stream));
  MLP_HIP(hipMemcpy(m.params, st.params.data(), kMlpP * 4, hipMemcpyHostToDevice));
  MLP_HIP(hipMemcpy(m.m, st.m.data(), kMlpP * 4, hipMemcpyHostToDevice));
  MLP_HIP(hipMemcpy(m.v, st.v.data(), kMlpP * 4, hipMemcpyHostToDevice));
  m.step = st.step;
}

namespace {

struct MlpCost final : CostModel {
  psc_mlp &m;
  explicit MlpCost(psc_mlp &m_) : m(m_) {}
  void predict_us(const float *feat, int64_t n, double *us) override {
    if (n <= 0) return;
    std::vector<float> y(n);
    mlp_predict(m, feat, n, y.data());
    for (int64_t i = 0; i < n; ++i) us[i] = std::exp(double(y[i]));
  }
};

}  // namespace

std::unique_ptr<CostModel> mlp_cost_model(const psc_mlp *m) {
  return std::make_unique<MlpCost>(*const_cast<psc_mlp *>(m));
}

}  // namespace psc

psc_mlp::~psc_mlp() {
  if (hipSetDevice(device) != hipSuccess) return;
  if (stream) (void)hipStreamSynchronize(stream);
  float *fl[] = {params, m, v, g, norm, x, t, z1, z2, y, dz1, dz2, dy};
  for (float *p : fl)
    if (p) (void)hipFree(p);
  if (idx) (void)hipFree(idx);
  if (stream) (void)hipStreamDestroy(stream);
}
