// Beam-width predictor training on the GPU: forward, gradient, Adam.
//
// Network: x = (f - mean) / scale (12 features), h1 = relu(W1 x + b1),
// h2 = relu(W2 h1 + b2), y = W3 . h2 + b3; loss = mean over the batch of
// (y - t)^2.  One wave per sample with one hidden unit per lane; each wave
// accumulates the gradient of the samples it visits in registers (lane j
// owns row j of W1 and W2 and entry j of b1, b2, W3), writes it to its own
// slice of a workspace, and a second kernel adds the slices in a fixed
// order, so the result does not depend on scheduling.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstring>
#include <mutex>

#include "../../include/esg.h"
#include "esg_kernels.h"
#include "esg_wave.h"

namespace {

using namespace esgk;

constexpr int kGradWaves = 512;                 // waves of the gradient kernel
constexpr int kSlice = kMlpWeights + 1;         // gradient + loss per wave

struct Act {
  float x[kFeat];
  float a1, h1, a2, h2, y;
};

__device__ __forceinline__ Act forward_one(const float* __restrict__ P, const float* f,
                                           float* lds_h1, int lane) {
  Act s;
#pragma unroll
  for (int i = 0; i < kFeat; i++) s.x[i] = (f[i] - P[kOffMu + i]) / P[kOffSd + i];
  float a1 = P[kOffB1 + lane];
#pragma unroll
  for (int i = 0; i < kFeat; i++) a1 = __builtin_fmaf(P[kOffW1 + lane * kFeat + i], s.x[i], a1);
  s.a1 = a1;
  s.h1 = a1 > 0.0f ? a1 : 0.0f;
  lds_h1[lane] = s.h1;
  wave_lds_sync();
  float a2 = P[kOffB2 + lane];
  for (int i = 0; i < kHidden; i++) a2 = __builtin_fmaf(P[kOffW2 + lane * kHidden + i], lds_h1[i], a2);
  s.a2 = a2;
  s.h2 = a2 > 0.0f ? a2 : 0.0f;
  float y = P[kOffW3 + lane] * s.h2;
#pragma unroll
  for (int m = 1; m < kWave; m <<= 1) y = y + xor_f(y, m, lane);
  s.y = y + P[kOffB3];
  return s;
}

__global__ __launch_bounds__(256) void mlp_forward_kernel(const float* __restrict__ P,
                                                          const float* __restrict__ F, int64_t B,
                                                          float* __restrict__ Y) {
  __shared__ float h1s[4][kHidden];
  const int lane = lane_id();
  const int w = threadIdx.x >> 6;
  for (int64_t b = (int64_t)blockIdx.x * 4 + w; b < B; b += (int64_t)gridDim.x * 4) {
    const Act s = forward_one(P, F + b * kFeat, h1s[w], lane);
    if (lane == 0) Y[b] = s.y;
    wave_lds_sync();
  }
}

__global__ __launch_bounds__(256) void mlp_grad_kernel(const float* __restrict__ P,
                                                       const float* __restrict__ F,
                                                       const float* __restrict__ T, int64_t B,
                                                       float* __restrict__ slices) {
  __shared__ float h1s[4][kHidden];
  __shared__ float g2s[4][kHidden];
  const int lane = lane_id();
  const int w = threadIdx.x >> 6;
  const int64_t wave = (int64_t)blockIdx.x * 4 + w;
  float gW1[kFeat], gW2[kHidden];
#pragma unroll
  for (int i = 0; i < kFeat; i++) gW1[i] = 0.0f;
#pragma unroll
  for (int i = 0; i < kHidden; i++) gW2[i] = 0.0f;
  float gb1 = 0.0f, gb2 = 0.0f, gW3 = 0.0f, gb3 = 0.0f, loss = 0.0f;
  const float inv_b = 1.0f / (float)B;
  for (int64_t b = wave; b < B; b += (int64_t)gridDim.x * 4) {
    const Act s = forward_one(P, F + b * kFeat, h1s[w], lane);
    const float err = s.y - T[b];
    loss += err * err * inv_b;
    const float gy = 2.0f * err * inv_b;
    gb3 += gy;
    gW3 = __builtin_fmaf(gy, s.h2, gW3);
    const float g2 = s.a2 > 0.0f ? gy * P[kOffW3 + lane] : 0.0f;   // dL/da2 of unit `lane`
    gb2 += g2;
#pragma unroll
    for (int i = 0; i < kHidden; i++) gW2[i] = __builtin_fmaf(g2, h1s[w][i], gW2[i]);
    g2s[w][lane] = g2;
    wave_lds_sync();
    float g1 = 0.0f;                                                   // dL/dh1 of unit `lane`
    for (int j = 0; j < kHidden; j++) g1 = __builtin_fmaf(P[kOffW2 + j * kHidden + lane], g2s[w][j], g1);
    g1 = s.a1 > 0.0f ? g1 : 0.0f;
    gb1 += g1;
#pragma unroll
    for (int i = 0; i < kFeat; i++) gW1[i] = __builtin_fmaf(g1, s.x[i], gW1[i]);
    wave_lds_sync();
  }
  float* out = slices + wave * kSlice;
#pragma unroll
  for (int i = 0; i < kFeat; i++) out[kOffW1 + lane * kFeat + i] = gW1[i];
  out[kOffB1 + lane] = gb1;
#pragma unroll
  for (int i = 0; i < kHidden; i++) out[kOffW2 + lane * kHidden + i] = gW2[i];
  out[kOffB2 + lane] = gb2;
  out[kOffW3 + lane] = gW3;
  if (lane == 0) {
    out[kOffB3] = gb3;
    out[kMlpWeights] = loss;
  }
  // the loss of the other lanes is identical (gy is wave-uniform): lane 0 only
}

// grad[j] = sum over waves (fixed order) of slice[w][j]; j < kSlice.
__global__ void mlp_reduce_kernel(const float* __restrict__ slices, int nwaves,
                                  float* __restrict__ grad, float* __restrict__ loss) {
  const int j = blockIdx.x * blockDim.x + threadIdx.x;
  if (j >= kSlice) return;
  float s = 0.0f;
  for (int w = 0; w < nwaves; w++) s += slices[(int64_t)w * kSlice + j];
  if (j < kMlpWeights) grad[j] = s;
  else if (loss) *loss = s;
}

__global__ void mlp_adam_kernel(float* __restrict__ P, const float* __restrict__ g,
                                float* __restrict__ m1, float* __restrict__ m2, float lr, float b1,
                                float b2, float eps, float c1, float c2) {
  const int j = blockIdx.x * blockDim.x + threadIdx.x;
  if (j >= kMlpWeights) return;
  const float gj = g[j];
  const float a = b1 * m1[j] + (1.0f - b1) * gj;
  const float v = b2 * m2[j] + (1.0f - b2) * gj * gj;
  m1[j] = a;
  m2[j] = v;
  P[j] -= lr * (a / c1) / (sqrtf(v / c2) + eps);
}

// Scratch of esg_mlp_grad_noalloc: the per-wave gradient slices, in a
// file-scope device array (one copy per GPU, held until the process ends).
// Host code never passes `scratch` itself to a kernel: its name on the host
// is a stand-in, not a device address; the device address is looked up
// once per device with hipGetSymbolAddress and kept in scratch_ptr.
constexpr size_t kScratchFloats = (size_t)kGradWaves * kSlice;   // 10.4 MB
__device__ __align__(256) float scratch[kScratchFloats];

constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
float* g_scratch_ptr[kMaxDevices] = {};

// Device address of the scratch array on the current device (null on error).
float* scratch_on_current_device() {
  int dev = -1;
  if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= kMaxDevices) {
    (void)hipGetLastError();
    return nullptr;
  }
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  if (!g_scratch_ptr[dev]) {
    void* p = nullptr;
    if (hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)) != hipSuccess || !p) {
      (void)hipGetLastError();
      return nullptr;
    }
    g_scratch_ptr[dev] = static_cast<float*>(p);
  }
  return g_scratch_ptr[dev];
}

}  // namespace

extern "C" {

int32_t esg_mlp_forward(const float* params, const float* feats, int64_t n, float* out,
                        void* stream) {
  if (!params || (n > 0 && (!feats || !out)) || n < 0) return ESG_EINVAL;
  if (n == 0) return ESG_OK;
  const int64_t grid = std::min<int64_t>((n + 3) / 4, 65536);
  mlp_forward_kernel<<<(unsigned)grid, 256, 0, static_cast<hipStream_t>(stream)>>>(params, feats,
                                                                                 n, out);
  return hipGetLastError() == hipSuccess ? ESG_OK : ESG_EHIP;
}

int32_t esg_mlp_grad(const float* params, const float* feats, const float* target, int64_t n,
                     float* grad, float* loss, float* workspace, void* stream) {
  if (!params || !feats || !target || !grad || !workspace || n < 1) return ESG_EINVAL;
  hipStream_t s = static_cast<hipStream_t>(stream);
  mlp_grad_kernel<<<kGradWaves / 4, 256, 0, s>>>(params, feats, target, n, workspace);
  mlp_reduce_kernel<<<(kSlice + 255) / 256, 256, 0, s>>>(workspace, kGradWaves, grad, loss);
  return hipGetLastError() == hipSuccess ? ESG_OK : ESG_EHIP;
}

int32_t esg_mlp_grad_noalloc(const float* params, const float* feats, const float* target,
                             int64_t n, float* grad, float* loss, void* stream) {
  if (!params || !feats || !target || !grad || n < 1) return ESG_EINVAL;
  // the scratch holds one slice per gradient wave whatever n is; every call
  // rewrites all of it, so nothing has to be cleared between calls
  static_assert(kScratchFloats == (size_t)ESG_MLP_WORKSPACE_FLOATS, "scratch size");
  float* ws = scratch_on_current_device();
  if (!ws) return ESG_EHIP;
  hipStream_t s = static_cast<hipStream_t>(stream);
  mlp_grad_kernel<<<kGradWaves / 4, 256, 0, s>>>(params, feats, target, n, ws);
  mlp_reduce_kernel<<<(kSlice + 255) / 256, 256, 0, s>>>(ws, kGradWaves, grad, loss);
  return hipGetLastError() == hipSuccess ? ESG_OK : ESG_EHIP;
}

int32_t esg_mlp_adam(float* params, const float* grad, float* m1, float* m2, int64_t step,
                     float lr, void* stream) {
  if (!params || !grad || !m1 || !m2 || step < 1 || !(lr > 0.0f)) return ESG_EINVAL;
  const float b1 = 0.9f, b2 = 0.999f, eps = 1e-8f;
  // bias corrections 1 - beta^t in double: in float32 the subtraction
  // cancels (1 - 0.999^2 keeps only about 3 significant digits)
  const float c1 = (float)(1.0 - pow((double)b1, (double)step));
  const float c2 = (float)(1.0 - pow((double)b2, (double)step));
  mlp_adam_kernel<<<(kMlpWeights + 255) / 256, 256, 0, static_cast<hipStream_t>(stream)>>>(
      params, grad, m1, m2, lr, b1, b2, eps, c1, c2);
  return hipGetLastError() == hipSuccess ? ESG_OK : ESG_EHIP;
}

}  // extern "C"
