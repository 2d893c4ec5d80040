// The learned selector's network, 8 -> 64 -> 64 -> 2 with tanh hidden
// layers, FP32 (gfx950): forward, backward, weight gradients and Adam.
//
// Parameters, one FP32 vector: W1 (64 x 8), b1 (64), W2 (64 x 64), b2 (64),
// W3 (2 x 64), b3 (2).  Loss: mean over the B x 2 outputs of (y - t)^2.
// The per-sample passes keep one sample per thread with the weights in LDS;
// the weight gradients sum over the samples in a fixed order (chunked, then
// reduced), so a gradient is the same from run to run.
#include <hip/hip_runtime.h>

#include "phiq_internal.h"

namespace phiq {
namespace {

constexpr int F = kMlpIn, H = kMlpHidden, O = kMlpOut;
constexpr int OW1 = 0, OB1 = OW1 + H * F, OW2 = OB1 + H, OB2 = OW2 + H * H, OW3 = OB2 + H, OB3 = OW3 + O * H;
static_assert(OB3 + O == kMlpParams, "parameter layout");

__device__ void load_weights(const float* __restrict__ w, float* s) {
  for (int i = threadIdx.x; i < kMlpParams; i += blockDim.x) s[i] = w[i];
  __syncthreads();
}

// y = W3 tanh(W2 tanh(W1 x + b1) + b2) + b3 for one sample per thread
__global__ __launch_bounds__(256) void mlp_forward_kernel(const float* __restrict__ w, const float* __restrict__ X,
                                                          int B, float* __restrict__ H1, float* __restrict__ H2,
                                                          float* __restrict__ Y) {
  __shared__ float s[kMlpParams];
  load_weights(w, s);
  const int b = blockIdx.x * blockDim.x + threadIdx.x;
  if (b >= B) return;
  float x[F], h1[H];
  for (int k = 0; k < F; ++k) x[k] = X[(long long)b * F + k];
  for (int i = 0; i < H; ++i) {
    float z = s[OB1 + i];
    for (int k = 0; k < F; ++k) z += s[OW1 + i * F + k] * x[k];
    h1[i] = tanhf(z);
    if (H1) H1[(long long)b * H + i] = h1[i];
  }
  float y[O];
  for (int o = 0; o < O; ++o) y[o] = s[OB3 + o];
  for (int i = 0; i < H; ++i) {
    float z = s[OB2 + i];
    for (int j = 0; j < H; ++j) z += s[OW2 + i * H + j] * h1[j];
    const float h2 = tanhf(z);
    if (H2) H2[(long long)b * H + i] = h2;
    for (int o = 0; o < O; ++o) y[o] += s[OW3 + o * H + i] * h2;
  }
  for (int o = 0; o < O; ++o) Y[(long long)b * O + o] = y[o];
}

// Per sample: dY = 2 (y - t) / (B O), dZ2 = (W3^T dY) (1 - h2^2),
// dZ1 = (W2^T dZ2) (1 - h1^2); block sums of the squared error.
__global__ __launch_bounds__(256) void mlp_backward_kernel(const float* __restrict__ w, const float* __restrict__ T,
                                                           const float* __restrict__ H1, const float* __restrict__ H2,
                                                           const float* __restrict__ Y, int B,
                                                           float* __restrict__ dY, float* __restrict__ dZ2,
                                                           float* __restrict__ dZ1, double* __restrict__ loss_part) {
  __shared__ float s[kMlpParams];
  __shared__ double red[256];
  load_weights(w, s);
  const int b = blockIdx.x * blockDim.x + threadIdx.x;
  double se = 0.0;
  if (b < B) {
    float dy[O];
    for (int o = 0; o < O; ++o) {
      const float e = Y[(long long)b * O + o] - T[(long long)b * O + o];
      se += (double)e * e;
      dy[o] = 2.0f * e / (float)((long long)B * O);
      dY[(long long)b * O + o] = dy[o];
    }
    float dz2[H];
    for (int i = 0; i < H; ++i) {
      const float h2 = H2[(long long)b * H + i];
      float g = 0.0f;
      for (int o = 0; o < O; ++o) g += s[OW3 + o * H + i] * dy[o];
      dz2[i] = g * (1.0f - h2 * h2);
      dZ2[(long long)b * H + i] = dz2[i];
    }
    for (int j = 0; j < H; ++j) {
      const float h1 = H1[(long long)b * H + j];
      float g = 0.0f;
      for (int i = 0; i < H; ++i) g += s[OW2 + i * H + j] * dz2[i];
      dZ1[(long long)b * H + j] = g * (1.0f - h1 * h1);
    }
  }
  red[threadIdx.x] = se;
  __syncthreads();
  for (int k = 128; k > 0; k >>= 1) {
    if (threadIdx.x < k) red[threadIdx.x] += red[threadIdx.x + k];
    __syncthreads();
  }
  if (threadIdx.x == 0 && loss_part) loss_part[blockIdx.x] = red[0];
}

// Partial gradient of parameter `q` over samples [c * per, (c+1) * per).
__global__ __launch_bounds__(256) void mlp_wgrad_kernel(const float* __restrict__ X, const float* __restrict__ H1,
                                                        const float* __restrict__ H2, const float* __restrict__ dZ1,
                                                        const float* __restrict__ dZ2, const float* __restrict__ dY,
                                                        int B, int per, double* __restrict__ part) {
  const int q = blockIdx.x * blockDim.x + threadIdx.x;
  if (q >= kMlpParams) return;
  const int c = blockIdx.y;
  const int b0 = c * per, b1 = min(B, b0 + per);
  // gradient of q = sum_b  g[b][gi] * a[b][ai]  (a = 1 for a bias)
  const float* g;
  const float* a = nullptr;
  int gs, gi, as = 0, ai = 0;
  if (q < OB1) { g = dZ1; gs = H; gi = (q - OW1) / F; a = X; as = F; ai = (q - OW1) % F; }
  else if (q < OW2) { g = dZ1; gs = H; gi = q - OB1; }
  else if (q < OB2) { g = dZ2; gs = H; gi = (q - OW2) / H; a = H1; as = H; ai = (q - OW2) % H; }
  else if (q < OW3) { g = dZ2; gs = H; gi = q - OB2; }
  else if (q < OB3) { g = dY; gs = O; gi = (q - OW3) / H; a = H2; as = H; ai = (q - OW3) % H; }
  else { g = dY; gs = O; gi = q - OB3; }
  double acc = 0.0;
  if (a) {
    for (int b = b0; b < b1; ++b) acc += (double)g[(long long)b * gs + gi] * (double)a[(long long)b * as + ai];
  } else {
    for (int b = b0; b < b1; ++b) acc += (double)g[(long long)b * gs + gi];
  }
  part[(long long)c * kMlpParams + q] = acc;
}

__global__ void mlp_reduce_kernel(const double* __restrict__ part, int chunks, float* __restrict__ grad) {
  const int q = blockIdx.x * blockDim.x + threadIdx.x;
  if (q >= kMlpParams) return;
  double acc = 0.0;
  for (int c = 0; c < chunks; ++c) acc += part[(long long)c * kMlpParams + q];
  grad[q] = (float)acc;
}

// Adam (Kingma and Ba): m = b1 m + (1 - b1) g, v = b2 v + (1 - b2) g^2,
// w -= lr (m / (1 - b1^t)) / (sqrt(v / (1 - b2^t)) + eps).
__global__ void mlp_adam_kernel(float* __restrict__ w, const float* __restrict__ g, float* __restrict__ m,
                                float* __restrict__ v, float lr, float b1, float b2, float eps, float c1, float c2) {
  const int q = blockIdx.x * blockDim.x + threadIdx.x;
  if (q >= kMlpParams) return;
  const float gq = g[q];
  const float mq = b1 * m[q] + (1.0f - b1) * gq;
  const float vq = b2 * v[q] + (1.0f - b2) * gq * gq;
  m[q] = mq;
  v[q] = vq;
  w[q] -= lr * (mq / c1) / (sqrtf(vq / c2) + eps);
}

inline int cdiv(long long a, long long b) { return (int)((a + b - 1) / b); }

}  // namespace

int launch_mlp_forward(const float* w, const float* X, int B, float* H1, float* H2, float* Y, void* stream) {
  hipLaunchKernelGGL(mlp_forward_kernel, dim3(cdiv(B, 256)), dim3(256), 0, (hipStream_t)stream, w, X, B, H1, H2, Y);
  return hipGetLastError();
}

int launch_mlp_backward(const float* w, const float* T, const float* H1, const float* H2, const float* Y, int B,
                        float* dY, float* dZ2, float* dZ1, double* loss_part, void* stream) {
  hipLaunchKernelGGL(mlp_backward_kernel, dim3(cdiv(B, 256)), dim3(256), 0, (hipStream_t)stream, w, T, H1, H2, Y, B,
                     dY, dZ2, dZ1, loss_part);
  return hipGetLastError();
}

int launch_mlp_wgrad(const float* X, const float* H1, const float* H2, const float* dZ1, const float* dZ2,
                     const float* dY, int B, int chunks, double* part, float* grad, void* stream) {
  const int per = cdiv(B, chunks);
  hipLaunchKernelGGL(mlp_wgrad_kernel, dim3(cdiv(kMlpParams, 256), chunks), dim3(256), 0, (hipStream_t)stream, X, H1,
                     H2, dZ1, dZ2, dY, B, per, part);
  hipLaunchKernelGGL(mlp_reduce_kernel, dim3(cdiv(kMlpParams, 256)), dim3(256), 0, (hipStream_t)stream, part, chunks,
                     grad);
  return hipGetLastError();
}

int launch_mlp_adam(float* w, const float* g, float* m, float* v, float lr, float b1, float b2, float eps, int step,
                    void* stream) {
  const float c1 = 1.0f - powf(b1, (float)step), c2 = 1.0f - powf(b2, (float)step);
  hipLaunchKernelGGL(mlp_adam_kernel, dim3(cdiv(kMlpParams, 256)), dim3(256), 0, (hipStream_t)stream, w, g, m, v, lr,
                     b1, b2, eps, c1, c2);
  return hipGetLastError();
}

}  // namespace phiq
