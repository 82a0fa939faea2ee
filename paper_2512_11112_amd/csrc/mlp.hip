// FP32 MLP cost model of the learned dispatcher: 7 -> 64 -> 64 -> 64 -> 2 with
// ReLU on the hidden layers, trained by minibatch Adam on the mean squared
// error.  Forward: one thread per sample, parameters staged in LDS.  Backward:
// per-sample deltas, then one thread per parameter summing over the batch (no
// atomics, so gradients are deterministic).
#include <string.h>

#include <algorithm>
#include <numeric>
#include <random>
#include <vector>

#include "ctx.h"

namespace spdz {

constexpr int IN = SPDZ_MLP_IN, HID = SPDZ_MLP_HID, OUT = SPDZ_MLP_OUT;
// parameter offsets
constexpr int OW1 = 0, OB1 = OW1 + HID * IN, OW2 = OB1 + HID, OB2 = OW2 + HID * HID, OW3 = OB2 + HID,
              OB3 = OW3 + HID * HID, OW4 = OB3 + HID, OB4 = OW4 + OUT * HID, NPARAM = OB4 + OUT;
static_assert(NPARAM == SPDZ_MLP_NPARAM, "parameter count");

__global__ __launch_bounds__(256) void k_mlp_forward(const float *__restrict__ W, const float *__restrict__ X,
                                                     int64_t B, float *__restrict__ Y, float *__restrict__ acts) {
  __shared__ float w[NPARAM];
  for (int i = threadIdx.x; i < NPARAM; i += 256) w[i] = W[i];
  __syncthreads();
  const int64_t b = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (b >= B) return;
  float x[IN], h1[HID], h2[HID];
#pragma unroll
  for (int k = 0; k < IN; k++) x[k] = X[b * IN + k];
#pragma unroll 4
  for (int j = 0; j < HID; j++) {
    float s = w[OB1 + j];
#pragma unroll
    for (int k = 0; k < IN; k++) s = fmaf(w[OW1 + j * IN + k], x[k], s);
    h1[j] = fmaxf(s, 0.f);
  }
#pragma unroll 4
  for (int j = 0; j < HID; j++) {
    float s = w[OB2 + j];
#pragma unroll
    for (int k = 0; k < HID; k++) s = fmaf(w[OW2 + j * HID + k], h1[k], s);
    h2[j] = fmaxf(s, 0.f);
  }
  if (acts) {
    for (int j = 0; j < HID; j++) {
      acts[(0 * B + b) * HID + j] = h1[j];
      acts[(1 * B + b) * HID + j] = h2[j];
    }
  }
  // layer 3 reuses h1 as storage
#pragma unroll 4
  for (int j = 0; j < HID; j++) {
    float s = w[OB3 + j];
#pragma unroll
    for (int k = 0; k < HID; k++) s = fmaf(w[OW3 + j * HID + k], h2[k], s);
    h1[j] = fmaxf(s, 0.f);
  }
  if (acts)
    for (int j = 0; j < HID; j++) acts[(2 * B + b) * HID + j] = h1[j];
#pragma unroll
  for (int o = 0; o < OUT; o++) {
    float s = w[OB4 + o];
#pragma unroll
    for (int k = 0; k < HID; k++) s = fmaf(w[OW4 + o * HID + k], h1[k], s);
    Y[b * OUT + o] = s;
  }
}

// per-sample deltas of the pre-activations: D [3][B][64] (layers 1..3); dY is the output delta
__global__ __launch_bounds__(256) void k_mlp_deltas(const float *__restrict__ W, const float *__restrict__ acts,
                                                    const float *__restrict__ dY, int64_t B, float *__restrict__ D) {
  __shared__ float w[NPARAM];
  for (int i = threadIdx.x; i < NPARAM; i += 256) w[i] = W[i];
  __syncthreads();
  const int64_t b = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (b >= B) return;
  float dn[HID], dc[HID];
  // layer 3: dh3 = W4^T dY, masked by h3 > 0
  for (int k = 0; k < HID; k++) {
    float s = 0.f;
#pragma unroll
    for (int o = 0; o < OUT; o++) s = fmaf(w[OW4 + o * HID + k], dY[b * OUT + o], s);
    dc[k] = acts[(2 * B + b) * HID + k] > 0.f ? s : 0.f;
    D[(2 * B + b) * HID + k] = dc[k];
  }
  // layer 2: dh2 = W3^T d3
  for (int k = 0; k < HID; k++) {
    float s = 0.f;
    for (int j = 0; j < HID; j++) s = fmaf(w[OW3 + j * HID + k], dc[j], s);
    dn[k] = acts[(1 * B + b) * HID + k] > 0.f ? s : 0.f;
    D[(1 * B + b) * HID + k] = dn[k];
  }
  // layer 1: dh1 = W2^T d2
  for (int k = 0; k < HID; k++) {
    float s = 0.f;
    for (int j = 0; j < HID; j++) s = fmaf(w[OW2 + j * HID + k], dn[j], s);
    D[(0 * B + b) * HID + k] = acts[(0 * B + b) * HID + k] > 0.f ? s : 0.f;
  }
}

// one thread per parameter: sum over the batch of delta (x) input
__global__ __launch_bounds__(256) void k_mlp_wgrad(const float *__restrict__ X, const float *__restrict__ acts,
                                                   const float *__restrict__ D, const float *__restrict__ dY, int64_t B,
                                                   float *__restrict__ dW) {
  const int p = blockIdx.x * 256 + threadIdx.x;
  if (p >= NPARAM) return;
  float s = 0.f;
  if (p < OB1) {
    const int j = p / IN, k = p % IN;
    for (int64_t b = 0; b < B; b++) s = fmaf(D[(0 * B + b) * HID + j], X[b * IN + k], s);
  } else if (p < OW2) {
    const int j = p - OB1;
    for (int64_t b = 0; b < B; b++) s += D[(0 * B + b) * HID + j];
  } else if (p < OB2) {
    const int j = (p - OW2) / HID, k = (p - OW2) % HID;
    for (int64_t b = 0; b < B; b++) s = fmaf(D[(1 * B + b) * HID + j], acts[(0 * B + b) * HID + k], s);
  } else if (p < OW3) {
    const int j = p - OB2;
    for (int64_t b = 0; b < B; b++) s += D[(1 * B + b) * HID + j];
  } else if (p < OB3) {
    const int j = (p - OW3) / HID, k = (p - OW3) % HID;
    for (int64_t b = 0; b < B; b++) s = fmaf(D[(2 * B + b) * HID + j], acts[(1 * B + b) * HID + k], s);
  } else if (p < OW4) {
    const int j = p - OB3;
    for (int64_t b = 0; b < B; b++) s += D[(2 * B + b) * HID + j];
  } else if (p < OB4) {
    const int o = (p - OW4) / HID, k = (p - OW4) % HID;
    for (int64_t b = 0; b < B; b++) s = fmaf(dY[b * OUT + o], acts[(2 * B + b) * HID + k], s);
  } else {
    const int o = p - OB4;
    for (int64_t b = 0; b < B; b++) s += dY[b * OUT + o];
  }
  dW[p] = s;
}

__global__ __launch_bounds__(256) void k_mlp_adam(float *W, const float *dW, float *m, float *v, float lr, float b1,
                                                  float b2, float eps, float c1, float c2) {
  const int p = blockIdx.x * 256 + threadIdx.x;
  if (p >= NPARAM) return;
  const float g = dW[p];
  const float mm = b1 * m[p] + (1.f - b1) * g;
  const float vv = b2 * v[p] + (1.f - b2) * g * g;
  m[p] = mm;
  v[p] = vv;
  W[p] -= lr * (mm / c1) / (sqrtf(vv / c2) + eps);
}

// dY = 2 (Y - T) / (B * OUT): gradient of the mean squared error over the batch
__global__ __launch_bounds__(256) void k_mse_grad(const float *Y, const float *T, int64_t n, float scale, float *dY) {
  const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (i < n) dY[i] = scale * (Y[i] - T[i]);
}

__global__ __launch_bounds__(256) void k_gather_rows(const float *src, const int32_t *idx, int64_t B, int width,
                                                     float *dst) {
  const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (i < B * width) dst[i] = src[(int64_t)idx[i / width] * width + i % width];
}

static unsigned blocks(int64_t n) { return (unsigned)((n + 255) / 256); }

spdz_status mlp_forward_launch(hipStream_t st, const float *W, const float *X, int64_t B, float *Y, float *acts) {
  if (B <= 0) return SPDZ_OK;
  hipLaunchKernelGGL(k_mlp_forward, dim3(blocks(B)), dim3(256), 0, st, W, X, B, Y, acts);
  return hip_status(hipGetLastError());
}

}  // namespace spdz

using namespace spdz;

extern "C" {

spdz_status spdz_mlp_forward(void *stream, const float *W, const float *X, int64_t B, float *Y, float *acts) {
  if (!W || !X || !Y || B < 0) return SPDZ_E_INVAL;
  return mlp_forward_launch((hipStream_t)stream, W, X, B, Y, acts);
}

spdz_status spdz_mlp_backward(void *stream, const float *W, const float *X, const float *acts, const float *dY,
                              int64_t B, float *dW) {
  if (!W || !X || !acts || !dY || !dW || B < 1) return SPDZ_E_INVAL;
  hipStream_t st = (hipStream_t)stream;
  float *D = nullptr;
  if (hipMallocAsync((void **)&D, (size_t)3 * B * HID * sizeof(float), st) != hipSuccess) return SPDZ_E_NOMEM;
  hipLaunchKernelGGL(k_mlp_deltas, dim3(blocks(B)), dim3(256), 0, st, W, acts, dY, B, D);
  hipLaunchKernelGGL(k_mlp_wgrad, dim3(blocks(NPARAM)), dim3(256), 0, st, X, acts, D, dY, B, dW);
  spdz_status s = hip_status(hipGetLastError());
  (void)hipFreeAsync(D, st);
  return s;
}

spdz_status spdz_mlp_adam(void *stream, float *W, const float *dW, float *m, float *v, int64_t t, float lr, float beta1,
                          float beta2, float eps) {
  if (!W || !dW || !m || !v || t < 1) return SPDZ_E_INVAL;
  const float c1 = 1.f - powf(beta1, (float)t), c2 = 1.f - powf(beta2, (float)t);
  hipLaunchKernelGGL(k_mlp_adam, dim3(blocks(NPARAM)), dim3(256), 0, (hipStream_t)stream, W, dW, m, v, lr, beta1, beta2,
                     eps, c1, c2);
  return hip_status(hipGetLastError());
}

spdz_status spdz_mlp_train(void *stream, float *W, const float *X, const float *T, int64_t N, int epochs, int batch,
                           float lr, uint64_t seed, float *loss_per_epoch) {
  if (!W || !X || !T || N < 1 || epochs < 1 || batch < 1) return SPDZ_E_INVAL;
  hipStream_t st = (hipStream_t)stream;
  const int64_t Bm = std::min<int64_t>(batch, N);
  float *buf = nullptr;
  int32_t *d_idx = nullptr;
  const size_t nb = (size_t)Bm * IN + (size_t)Bm * OUT * 3 + (size_t)3 * Bm * HID + 3 * (size_t)NPARAM +
                    (size_t)N * OUT;
  if (hipMalloc((void **)&buf, nb * sizeof(float)) != hipSuccess) return SPDZ_E_NOMEM;
  if (hipMalloc((void **)&d_idx, (size_t)N * sizeof(int32_t)) != hipSuccess) {
    (void)hipFree(buf);
    return SPDZ_E_NOMEM;
  }
  float *xb = buf, *tb = xb + Bm * IN, *yb = tb + Bm * OUT, *dy = yb + Bm * OUT, *acts = dy + Bm * OUT,
        *dW = acts + 3 * Bm * HID, *m = dW + NPARAM, *v = m + NPARAM, *yall = v + NPARAM;
  spdz_status s = hip_status(hipMemsetAsync(m, 0, 2 * NPARAM * sizeof(float), st));
  std::vector<int32_t> order(N);
  std::iota(order.begin(), order.end(), 0);
  std::mt19937_64 rng(seed);
  std::vector<float> yh((size_t)N * OUT), th((size_t)N * OUT);
  if (s == SPDZ_OK && loss_per_epoch)
    s = hip_status(hipMemcpyAsync(th.data(), T, th.size() * sizeof(float), hipMemcpyDeviceToHost, st));
  int64_t step = 0;
  for (int ep = 0; ep < epochs && s == SPDZ_OK; ep++) {
    std::shuffle(order.begin(), order.end(), rng);
    s = hip_status(hipMemcpyAsync(d_idx, order.data(), (size_t)N * sizeof(int32_t), hipMemcpyHostToDevice, st));
    for (int64_t b0 = 0; b0 + Bm <= N && s == SPDZ_OK; b0 += Bm) {
      hipLaunchKernelGGL(k_gather_rows, dim3(blocks(Bm * IN)), dim3(256), 0, st, X, d_idx + b0, Bm, IN, xb);
      hipLaunchKernelGGL(k_gather_rows, dim3(blocks(Bm * OUT)), dim3(256), 0, st, T, d_idx + b0, Bm, OUT, tb);
      s = mlp_forward_launch(st, W, xb, Bm, yb, acts);
      if (s != SPDZ_OK) break;
      hipLaunchKernelGGL(k_mse_grad, dim3(blocks(Bm * OUT)), dim3(256), 0, st, yb, tb, Bm * OUT,
                         2.f / (float)(Bm * OUT), dy);
      s = spdz_mlp_backward(st, W, xb, acts, dy, Bm, dW);
      if (s == SPDZ_OK) s = spdz_mlp_adam(st, W, dW, m, v, ++step, lr, 0.9f, 0.999f, 1e-8f);
    }
    if (s == SPDZ_OK && loss_per_epoch) {
      s = mlp_forward_launch(st, W, X, N, yall, nullptr);
      if (s == SPDZ_OK)
        s = hip_status(hipMemcpyAsync(yh.data(), yall, yh.size() * sizeof(float), hipMemcpyDeviceToHost, st));
      if (s == SPDZ_OK) s = hip_status(hipStreamSynchronize(st));
      double acc = 0;
      for (size_t i = 0; i < yh.size(); i++) acc += (double)(yh[i] - th[i]) * (yh[i] - th[i]);
      loss_per_epoch[ep] = (float)(acc / yh.size());
    }
  }
  if (hipStreamSynchronize(st) != hipSuccess && s == SPDZ_OK) s = SPDZ_E_HIP;
  (void)hipFree(buf);
  (void)hipFree(d_idx);
  return s;
}

}  // extern "C"
