// The small network behind the learned sample-count predictor: 64 structural features
// -> 128 (ReLU) -> 128 (ReLU) -> 2 outputs, bfloat16 weights, FP32 accumulation, with
// hand-written forward, backward and Adam kernels. The choice of the initial number of
// training states is left open by the paper (Sec. 3 and Sec. 5); what the outputs mean
// and how they are used is in learned.hip.
//
// Loss per row r (mean over the rows of a batch):
//   m_r * (y0 - t0)^2 / 2 + softplus(y1) - t1 * y1
// where m_r = 1 when the regression label t0 is finite (0 for rows with no label), and
// the second term is the binary cross-entropy of the logit y1 against t1 in [0, 1].
// The FP32 master weights are updated by Adam; the bfloat16 copy used by every forward
// and backward pass is refreshed (round to nearest even) after each step.
#include <algorithm>
#include <cmath>
#include <cstring>
#include <fstream>
#include <mutex>
#include <vector>

#include "mlp.h"

namespace qfs {
namespace {

constexpr int kRows = 32;  // rows of a batch per work-group
constexpr int kLossBlocks = 64;

__device__ __forceinline__ float bf(uint16_t h) { return __uint_as_float((uint32_t)h << 16); }

__host__ __device__ inline uint16_t f32_to_bf16(float f) {
  uint32_t u;
#ifdef __HIP_DEVICE_COMPILE__
  u = __float_as_uint(f);
#else
  std::memcpy(&u, &f, 4);
#endif
  if ((u & 0x7f800000u) == 0x7f800000u)  // inf stays inf, NaN stays NaN
    return (uint16_t)((u >> 16) | ((u & 0xffffu) ? 0x40u : 0u));
  u += 0x7fffu + ((u >> 16) & 1u);
  return (uint16_t)(u >> 16);
}

// Forward pass of kRows rows per work-group (thread j = hidden unit j). Keeps the
// pre-activations and activations for the backward pass when Z1 != nullptr.
__global__ __launch_bounds__(kMlpH) void k_mlp_forward(int B, const float *__restrict__ X,
                                                       const uint16_t *__restrict__ W,
                                                       float *Z1, float *A1, float *Z2, float *A2,
                                                       float *__restrict__ Y) {
  __shared__ float xs[kRows][kMlpF + 1];
  __shared__ float h[kRows][kMlpH + 1];
  const int r0 = blockIdx.x * kRows, j = threadIdx.x;
  const int rows = min(kRows, B - r0);
  for (int e = j; e < kRows * kMlpF; e += kMlpH) {
    const int r = e / kMlpF, f = e % kMlpF;
    xs[r][f] = r < rows ? X[(size_t)(r0 + r) * kMlpF + f] : 0.f;
  }
  __syncthreads();
  {
    float w[kMlpF];
#pragma unroll
    for (int f = 0; f < kMlpF; ++f) w[f] = bf(W[kMlpW1 + j * kMlpF + f]);
    const float b = bf(W[kMlpB1 + j]);
    for (int r = 0; r < kRows; ++r) {
      float z = b;
#pragma unroll
      for (int f = 0; f < kMlpF; ++f) z = fmaf(w[f], xs[r][f], z);
      const float a = fmaxf(z, 0.f);
      h[r][j] = a;
      if (Z1 && r < rows) {
        Z1[(size_t)(r0 + r) * kMlpH + j] = z;
        A1[(size_t)(r0 + r) * kMlpH + j] = a;
      }
    }
  }
  __syncthreads();
  float z2[kRows];
  {
    const float b = bf(W[kMlpB2 + j]);
#pragma unroll
    for (int r = 0; r < kRows; ++r) z2[r] = b;
    for (int k = 0; k < kMlpH; ++k) {
      const float wk = bf(W[kMlpW2 + j * kMlpH + k]);
#pragma unroll
      for (int r = 0; r < kRows; ++r) z2[r] = fmaf(wk, h[r][k], z2[r]);
    }
  }
  __syncthreads();
#pragma unroll
  for (int r = 0; r < kRows; ++r) {
    const float a = fmaxf(z2[r], 0.f);
    h[r][j] = a;
    if (Z1 && r < rows) {
      Z2[(size_t)(r0 + r) * kMlpH + j] = z2[r];
      A2[(size_t)(r0 + r) * kMlpH + j] = a;
    }
  }
  __syncthreads();
  for (int e = j; e < kRows * kMlpO; e += kMlpH) {
    const int r = e / kMlpO, o = e % kMlpO;
    if (r >= rows) continue;
    float y = bf(W[kMlpB3 + o]);
    for (int k = 0; k < kMlpH; ++k) y = fmaf(bf(W[kMlpW3 + o * kMlpH + k]), h[r][k], y);
    Y[(size_t)(r0 + r) * kMlpO + o] = y;
  }
}

// Output gradients and per-block loss sums.
__global__ void k_mlp_dy(int B, const float *__restrict__ Y, const float *__restrict__ T,
                         float *__restrict__ dY, float *__restrict__ loss_part) {
  __shared__ float red[256];
  float l = 0.f;
  for (int r = blockIdx.x * blockDim.x + threadIdx.x; r < B; r += gridDim.x * blockDim.x) {
    const float y0 = Y[r * kMlpO], y1 = Y[r * kMlpO + 1], t0 = T[r * kMlpO], t1 = T[r * kMlpO + 1];
    float d0 = 0.f;
    if (isfinite(t0)) {
      d0 = y0 - t0;
      l += 0.5f * d0 * d0;
    }
    const float p = 1.f / (1.f + expf(-y1));
    l += fmaxf(y1, 0.f) + log1pf(expf(-fabsf(y1))) - t1 * y1;
    dY[r * kMlpO] = d0 / (float)B;
    dY[r * kMlpO + 1] = (p - t1) / (float)B;
  }
  red[threadIdx.x] = l;
  __syncthreads();
  for (int s = blockDim.x / 2; s > 0; s >>= 1) {
    if (threadIdx.x < s) red[threadIdx.x] += red[threadIdx.x + s];
    __syncthreads();
  }
  if (threadIdx.x == 0) loss_part[blockIdx.x] = red[0];
}

// Backward pass of kRows rows per work-group: writes this block's gradient partial
// G[block][kMlpNP] (summed over blocks in a fixed order by k_mlp_sum).
__global__ __launch_bounds__(kMlpH) void k_mlp_backward(int B, const float *__restrict__ X,
                                                        const uint16_t *__restrict__ W,
                                                        const float *__restrict__ Z1,
                                                        const float *__restrict__ A1,
                                                        const float *__restrict__ Z2,
                                                        const float *__restrict__ A2,
                                                        const float *__restrict__ dY,
                                                        float *__restrict__ G) {
  __shared__ float dz2[kRows][kMlpH + 1];
  __shared__ float dz1[kRows][kMlpH + 1];
  __shared__ float act[kRows][kMlpH + 1];  // A1, then X
  __shared__ float dy[kRows][kMlpO];
  const int r0 = blockIdx.x * kRows, j = threadIdx.x;
  const int rows = min(kRows, B - r0);
  float *g = G + (size_t)blockIdx.x * kMlpNP;
  for (int e = j; e < kRows * kMlpO; e += kMlpH) {
    const int r = e / kMlpO, o = e % kMlpO;
    dy[r][o] = r < rows ? dY[(size_t)(r0 + r) * kMlpO + o] : 0.f;
  }
  for (int e = j; e < kRows * kMlpH; e += kMlpH) {
    const int r = e / kMlpH, k = e % kMlpH;
    act[r][k] = r < rows ? A1[(size_t)(r0 + r) * kMlpH + k] : 0.f;
  }
  __syncthreads();
  // output layer: dW3[o][j] = sum_r dy[r][o] A2[r][j]; dA2 -> dZ2 through the ReLU
  {
    const float w30 = bf(W[kMlpW3 + j]), w31 = bf(W[kMlpW3 + kMlpH + j]);
    float g0 = 0.f, g1 = 0.f;
    for (int r = 0; r < kRows; ++r) {
      const bool live = r < rows;
      const float a2 = live ? A2[(size_t)(r0 + r) * kMlpH + j] : 0.f;
      const float z2 = live ? Z2[(size_t)(r0 + r) * kMlpH + j] : 0.f;
      g0 = fmaf(dy[r][0], a2, g0);
      g1 = fmaf(dy[r][1], a2, g1);
      const float da = fmaf(dy[r][0], w30, dy[r][1] * w31);
      dz2[r][j] = z2 > 0.f ? da : 0.f;
    }
    g[kMlpW3 + j] = g0;
    g[kMlpW3 + kMlpH + j] = g1;
    if (j < kMlpO) {
      float s = 0.f;
      for (int r = 0; r < kRows; ++r) s += dy[r][j];
      g[kMlpB3 + j] = s;
    }
  }
  __syncthreads();
  // hidden layer 2: dW2[j][k] = sum_r dz2[r][j] A1[r][k]; dA1[r][j] = sum_i dz2[r][i] W2[i][j]
  {
    float db = 0.f;
    for (int r = 0; r < kRows; ++r) db += dz2[r][j];
    g[kMlpB2 + j] = db;
    for (int k = 0; k < kMlpH; ++k) {
      float s = 0.f;
#pragma unroll 8
      for (int r = 0; r < kRows; ++r) s = fmaf(dz2[r][j], act[r][k], s);
      g[kMlpW2 + j * kMlpH + k] = s;
    }
    float da[kRows];
#pragma unroll
    for (int r = 0; r < kRows; ++r) da[r] = 0.f;
    for (int i = 0; i < kMlpH; ++i) {
      const float w = bf(W[kMlpW2 + i * kMlpH + j]);
#pragma unroll
      for (int r = 0; r < kRows; ++r) da[r] = fmaf(dz2[r][i], w, da[r]);
    }
#pragma unroll
    for (int r = 0; r < kRows; ++r) {
      const float z1 = r < rows ? Z1[(size_t)(r0 + r) * kMlpH + j] : 0.f;
      dz1[r][j] = z1 > 0.f ? da[r] : 0.f;
    }
  }
  __syncthreads();
  for (int e = j; e < kRows * kMlpF; e += kMlpH) {
    const int r = e / kMlpF, f = e % kMlpF;
    act[r][f] = r < rows ? X[(size_t)(r0 + r) * kMlpF + f] : 0.f;
  }
  __syncthreads();
  // hidden layer 1: dW1[j][f] = sum_r dz1[r][j] X[r][f]
  {
    float db = 0.f;
    for (int r = 0; r < kRows; ++r) db += dz1[r][j];
    g[kMlpB1 + j] = db;
    for (int f = 0; f < kMlpF; ++f) {
      float s = 0.f;
#pragma unroll 8
      for (int r = 0; r < kRows; ++r) s = fmaf(dz1[r][j], act[r][f], s);
      g[kMlpW1 + j * kMlpF + f] = s;
    }
  }
}

__global__ void k_mlp_sum(int nblk, const float *__restrict__ G, float *__restrict__ out) {
  const int e = blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= kMlpNP) return;
  float s = 0.f;
  for (int b = 0; b < nblk; ++b) s += G[(size_t)b * kMlpNP + e];
  out[e] = s;
}

__global__ void k_mlp_adam(float *P, float *m, float *v, const float *__restrict__ grad, uint16_t *W,
                           float lr, float b1, float b2, float eps, float c1, float c2) {
  const int e = blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= kMlpNP) return;
  const float gr = grad[e];
  const float mm = b1 * m[e] + (1.f - b1) * gr;
  const float vv = b2 * v[e] + (1.f - b2) * gr * gr;
  m[e] = mm;
  v[e] = vv;
  const float p = P[e] - lr * (mm / c1) / (sqrtf(vv / c2) + eps);
  P[e] = p;
  W[e] = f32_to_bf16(p);
}

__global__ void k_mlp_round(const float *__restrict__ P, uint16_t *__restrict__ W) {
  const int e = blockIdx.x * blockDim.x + threadIdx.x;
  if (e < kMlpNP) W[e] = f32_to_bf16(P[e]);
}

// Gather rows idx[0..B) of X [*][F] and T [*][O] into contiguous batch buffers.
__global__ void k_mlp_gather(int B, const int32_t *__restrict__ idx, const float *__restrict__ X,
                             const float *__restrict__ T, float *__restrict__ xb, float *__restrict__ tb) {
  const int e = blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= B * kMlpF) return;
  const int r = e / kMlpF, f = e % kMlpF;
  const size_t src = (size_t)idx[r];
  xb[e] = X[src * kMlpF + f];
  if (f < kMlpO) tb[r * kMlpO + f] = T[src * kMlpO + f];
}

// ------------------------------------------------------------------ process-wide model
struct Model {
  std::mutex mu;
  bool ready = false;
  DevBuf P, W, m, v;
  int64_t steps = 0;
};
Model g_model;

struct Work {
  DevBuf Z1, A1, Z2, A2, Y, dY, G, Gsum, lossp, xb, tb;
  int cap = 0;
  int alloc(int B) {
    if (B <= cap) return QFS_OK;
    const size_t nblk = (size_t)(B + kRows - 1) / kRows;
    QFS_TRY(Z1.alloc(sizeof(float) * (size_t)B * kMlpH));
    QFS_TRY(A1.alloc(sizeof(float) * (size_t)B * kMlpH));
    QFS_TRY(Z2.alloc(sizeof(float) * (size_t)B * kMlpH));
    QFS_TRY(A2.alloc(sizeof(float) * (size_t)B * kMlpH));
    QFS_TRY(Y.alloc(sizeof(float) * (size_t)B * kMlpO));
    QFS_TRY(dY.alloc(sizeof(float) * (size_t)B * kMlpO));
    QFS_TRY(G.alloc(sizeof(float) * nblk * kMlpNP));
    QFS_TRY(Gsum.alloc(sizeof(float) * kMlpNP));
    QFS_TRY(lossp.alloc(sizeof(float) * kLossBlocks));
    QFS_TRY(xb.alloc(sizeof(float) * (size_t)B * kMlpF));
    QFS_TRY(tb.alloc(sizeof(float) * (size_t)B * kMlpO));
    cap = B;
    return QFS_OK;
  }
};
Work g_work;

int ensure_model() {
  if (g_model.ready) return QFS_OK;
  QFS_TRY(g_model.P.alloc(sizeof(float) * kMlpNP));
  QFS_TRY(g_model.W.alloc(sizeof(uint16_t) * kMlpNP));
  QFS_TRY(g_model.m.alloc(sizeof(float) * kMlpNP));
  QFS_TRY(g_model.v.alloc(sizeof(float) * kMlpNP));
  g_model.ready = true;
  return QFS_OK;
}

uint64_t splitmix(uint64_t &x) {
  x += 0x9E3779B97F4A7C15ull;
  uint64_t z = x;
  z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
  z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
  return z ^ (z >> 31);
}

int upload(const float *host, hipStream_t s) {
  QFS_HIP(hipMemcpyAsync(g_model.P.ptr, host, sizeof(float) * kMlpNP, hipMemcpyHostToDevice, s));
  hipLaunchKernelGGL(k_mlp_round, dim3((kMlpNP + 255) / 256), dim3(256), 0, s, g_model.P.as<float>(),
                     g_model.W.as<uint16_t>());
  QFS_HIP(hipGetLastError());
  QFS_TRY(launch_zero(g_model.m.ptr, sizeof(float) * kMlpNP, s));
  QFS_TRY(launch_zero(g_model.v.ptr, sizeof(float) * kMlpNP, s));
  QFS_HIP(hipStreamSynchronize(s));
  g_model.steps = 0;
  return QFS_OK;
}

int forward(int B, const float *X, bool keep, hipStream_t s) {
  const int nblk = (B + kRows - 1) / kRows;
  Work &w = g_work;
  hipLaunchKernelGGL(k_mlp_forward, dim3(nblk), dim3(kMlpH), 0, s, B, X, g_model.W.as<uint16_t>(),
                     keep ? w.Z1.as<float>() : nullptr, w.A1.as<float>(), w.Z2.as<float>(),
                     w.A2.as<float>(), w.Y.as<float>());
  QFS_HIP(hipGetLastError());
  return QFS_OK;
}

int gradient(int B, const float *X, const float *T, hipStream_t s) {
  Work &w = g_work;
  QFS_TRY(forward(B, X, true, s));
  hipLaunchKernelGGL(k_mlp_dy, dim3(kLossBlocks), dim3(256), 0, s, B, w.Y.as<float>(), T, w.dY.as<float>(),
                     w.lossp.as<float>());
  QFS_HIP(hipGetLastError());
  const int nblk = (B + kRows - 1) / kRows;
  hipLaunchKernelGGL(k_mlp_backward, dim3(nblk), dim3(kMlpH), 0, s, B, X, g_model.W.as<uint16_t>(),
                     w.Z1.as<float>(), w.A1.as<float>(), w.Z2.as<float>(), w.A2.as<float>(),
                     w.dY.as<float>(), w.G.as<float>());
  QFS_HIP(hipGetLastError());
  hipLaunchKernelGGL(k_mlp_sum, dim3((kMlpNP + 255) / 256), dim3(256), 0, s, nblk, w.G.as<float>(),
                     w.Gsum.as<float>());
  QFS_HIP(hipGetLastError());
  return QFS_OK;
}

int read_loss(int B, float *out, hipStream_t s) {
  float lp[kLossBlocks];
  QFS_HIP(hipMemcpyAsync(lp, g_work.lossp.ptr, sizeof(lp), hipMemcpyDeviceToHost, s));
  QFS_HIP(hipStreamSynchronize(s));
  double l = 0.0;
  for (int i = 0; i < kLossBlocks; ++i) l += lp[i];
  *out = (float)(l / B);
  return QFS_OK;
}

}  // namespace

int mlp_predict(int B, const float *features_dev, float *out_dev, hipStream_t s) {
  std::lock_guard<std::mutex> lk(g_model.mu);
  if (!g_model.ready) {
    set_error_detail("mlp: no weights (call qfs_mlp_init, qfs_mlp_set or qfs_mlp_load)");
    return QFS_EINVAL;
  }
  QFS_TRY(g_work.alloc(B));
  QFS_TRY(forward(B, features_dev, false, s));
  QFS_HIP(hipMemcpyAsync(out_dev, g_work.Y.ptr, sizeof(float) * kMlpO * B, hipMemcpyDeviceToDevice, s));
  QFS_HIP(hipStreamSynchronize(s));
  return QFS_OK;
}

}  // namespace qfs

using namespace qfs;

extern "C" {

int qfs_mlp_num_params(void) { return kMlpNP; }

int qfs_mlp_init(uint64_t seed) {
  std::lock_guard<std::mutex> lk(g_model.mu);
  QFS_TRY(ensure_model());
  // He-uniform weights from a SplitMix64 stream, zero biases
  std::vector<float> p(kMlpNP, 0.f);
  uint64_t x = seed;
  auto fill = [&](int off, int count, int fan_in) {
    const double lim = std::sqrt(6.0 / fan_in);
    for (int i = 0; i < count; ++i) {
      const double u = (double)(splitmix(x) >> 11) * 0x1.0p-53;
      p[off + i] = (float)((2.0 * u - 1.0) * lim);
    }
  };
  fill(kMlpW1, kMlpH * kMlpF, kMlpF);
  fill(kMlpW2, kMlpH * kMlpH, kMlpH);
  fill(kMlpW3, kMlpO * kMlpH, kMlpH);
  return upload(p.data(), nullptr);
}

int qfs_mlp_get(float *host_params) {
  std::lock_guard<std::mutex> lk(g_model.mu);
  if (!g_model.ready || !host_params) return set_error_detail("mlp: no weights"), QFS_EINVAL;
  QFS_HIP(hipMemcpy(host_params, g_model.P.ptr, sizeof(float) * kMlpNP, hipMemcpyDeviceToHost));
  return QFS_OK;
}

int qfs_mlp_set(const float *host_params) {
  std::lock_guard<std::mutex> lk(g_model.mu);
  if (!host_params) return QFS_EINVAL;
  for (int i = 0; i < kMlpNP; ++i)
    if (!std::isfinite(host_params[i])) return set_error_detail("mlp: non-finite weight"), QFS_EINVAL;
  QFS_TRY(ensure_model());
  return upload(host_params, nullptr);
}

int qfs_mlp_save(const char *path) {
  if (!path) return QFS_EINVAL;
  std::vector<float> p(kMlpNP);
  QFS_TRY(qfs_mlp_get(p.data()));
  std::ofstream f(path, std::ios::binary);
  if (!f) return set_error_detail(std::string("mlp: cannot write ") + path), QFS_EINVAL;
  f.write(kMlpMagic, 8);
  f.write(reinterpret_cast<const char *>(p.data()), sizeof(float) * kMlpNP);
  return f ? QFS_OK : QFS_EINVAL;
}

int qfs_mlp_load(const char *path) {
  if (!path) return QFS_EINVAL;
  std::ifstream f(path, std::ios::binary);
  if (!f) return set_error_detail(std::string("mlp: cannot read ") + path), QFS_EINVAL;
  char magic[8];
  f.read(magic, 8);
  if (!f || std::memcmp(magic, kMlpMagic, 8) != 0)
    return set_error_detail(std::string("mlp: not a weight file: ") + path), QFS_EINVAL;
  std::vector<float> p(kMlpNP);
  f.read(reinterpret_cast<char *>(p.data()), sizeof(float) * kMlpNP);
  if (!f) return set_error_detail(std::string("mlp: truncated weight file: ") + path), QFS_EINVAL;
  return qfs_mlp_set(p.data());
}

int qfs_mlp_forward(int32_t count, const float *features, float *out, void *hip_stream) {
  if (count < 1 || !features || !out) return QFS_EINVAL;
  return mlp_predict(count, features, out, static_cast<hipStream_t>(hip_stream));
}

int qfs_mlp_grad(int32_t count, const float *features, const float *targets, float *grad_host,
                 float *loss_host, void *hip_stream) {
  std::lock_guard<std::mutex> lk(g_model.mu);
  if (count < 1 || !features || !targets) return QFS_EINVAL;
  if (!g_model.ready) return set_error_detail("mlp: no weights"), QFS_EINVAL;
  hipStream_t s = static_cast<hipStream_t>(hip_stream);
  QFS_TRY(g_work.alloc(count));
  QFS_TRY(gradient(count, features, targets, s));
  if (grad_host)
    QFS_HIP(hipMemcpyAsync(grad_host, g_work.Gsum.ptr, sizeof(float) * kMlpNP, hipMemcpyDeviceToHost, s));
  float l = 0.f;
  QFS_TRY(read_loss(count, &l, s));
  if (loss_host) *loss_host = l;
  return QFS_OK;
}

int qfs_mlp_train(int32_t count, const float *features, const float *targets, int32_t epochs,
                  int32_t batch, float lr, uint64_t seed, float *epoch_loss, void *hip_stream) {
  std::lock_guard<std::mutex> lk(g_model.mu);
  if (count < 1 || epochs < 1 || batch < 1 || batch > count || !features || !targets || !(lr > 0.f))
    return set_error_detail("mlp_train: bad arguments"), QFS_EINVAL;
  if (!g_model.ready) return set_error_detail("mlp: no weights"), QFS_EINVAL;
  hipStream_t s = static_cast<hipStream_t>(hip_stream);
  QFS_TRY(g_work.alloc(batch));
  DevBuf perm;
  QFS_TRY(perm.alloc(sizeof(int32_t) * (size_t)count));
  std::vector<int32_t> order(count);
  uint64_t x = seed;
  const float b1 = 0.9f, b2 = 0.999f;
  for (int ep = 0; ep < epochs; ++ep) {
    for (int i = 0; i < count; ++i) order[i] = i;
    for (int i = count - 1; i > 0; --i) std::swap(order[i], order[splitmix(x) % (uint64_t)(i + 1)]);
    QFS_HIP(hipMemcpyAsync(perm.ptr, order.data(), sizeof(int32_t) * count, hipMemcpyHostToDevice, s));
    double sum = 0.0;
    int nb = 0;
    for (int b0 = 0; b0 + batch <= count; b0 += batch) {
      hipLaunchKernelGGL(k_mlp_gather, dim3((batch * kMlpF + 255) / 256), dim3(256), 0, s, batch,
                         perm.as<int32_t>() + b0, features, targets, g_work.xb.as<float>(),
                         g_work.tb.as<float>());
      QFS_HIP(hipGetLastError());
      QFS_TRY(gradient(batch, g_work.xb.as<float>(), g_work.tb.as<float>(), s));
      ++g_model.steps;
      const float c1 = 1.f - std::pow(b1, (float)g_model.steps);
      const float c2 = 1.f - std::pow(b2, (float)g_model.steps);
      hipLaunchKernelGGL(k_mlp_adam, dim3((kMlpNP + 255) / 256), dim3(256), 0, s, g_model.P.as<float>(),
                         g_model.m.as<float>(), g_model.v.as<float>(), g_work.Gsum.as<float>(),
                         g_model.W.as<uint16_t>(), lr, b1, b2, 1e-8f, c1, c2);
      QFS_HIP(hipGetLastError());
      if (epoch_loss) {
        float l = 0.f;
        QFS_TRY(read_loss(batch, &l, s));
        sum += l;
      }
      ++nb;
    }
    if (epoch_loss) epoch_loss[ep] = (float)(sum / std::max(1, nb));
  }
  QFS_HIP(hipStreamSynchronize(s));
  return QFS_OK;
}

}  // extern "C"
