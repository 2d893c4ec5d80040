// Host side of the learned (l, m) selector: training driver over the HIP
// kernels of mlp.hip, the host forward pass used while planning, and the
// judge that accepts, corrects or rejects the network's choice with the a
// priori bound of Thm 3.2 (Algorithm setup_quadrature stays the fallback).
#include <algorithm>
#include <cmath>
#include <cstring>
#include <vector>

#include <hip/hip_runtime_api.h>

#include "phiq_internal.h"

#define PHIQ_TRY(x)                  \
  do {                               \
    const phiq_status s_ = (x);      \
    if (s_ != PHIQ_OK) return s_;    \
  } while (0)
#define PHIQ_HIP(x)                  \
  do {                               \
    if ((x) != hipSuccess) {         \
      (void)hipGetLastError();       \
      return PHIQ_ERR_HIP;           \
    }                                \
  } while (0)

namespace phiq {

void mlp_predict_host(const float* w, const float x[kMlpIn], float y[kMlpOut]) {
  constexpr int F = kMlpIn, H = kMlpHidden, O = kMlpOut;
  const float* W1 = w;
  const float* b1 = W1 + H * F;
  const float* W2 = b1 + H;
  const float* b2 = W2 + H * H;
  const float* W3 = b2 + H;
  const float* b3 = W3 + O * H;
  float h1[H];
  for (int i = 0; i < H; ++i) {
    float z = b1[i];
    for (int k = 0; k < F; ++k) z += W1[i * F + k] * x[k];
    h1[i] = std::tanh(z);
  }
  for (int o = 0; o < O; ++o) y[o] = b3[o];
  for (int i = 0; i < H; ++i) {
    float z = b2[i];
    for (int j = 0; j < H; ++j) z += W2[i * H + j] * h1[j];
    const float h2 = std::tanh(z);
    for (int o = 0; o < O; ++o) y[o] += W3[o * H + i] * h2;
  }
}

namespace {

// The network's 8 inputs for this problem.
void mlp_features(const phiq_kron_op* op, const double* norms, double t, int p, double tol, float x[kMlpIn]) {
  int nmax = 1;
  for (int d = 0; d < op->dim; ++d) nmax = std::max(nmax, op->n[d]);
  for (int d = 0; d < 3; ++d) x[d] = (d < op->dim) ? (float)std::log10(std::max(norms[d], 1e-300)) : -3.0f;
  x[3] = (float)(nmax / 256.0);
  x[4] = (float)op->dim;
  x[5] = (float)p;
  x[6] = (float)std::log10(std::fabs(t));
  x[7] = (float)std::log10(tol);
}

}  // namespace

bool mlp_choose(const float* w, const phiq_kron_op* op, const double* norms, double t, int p, double tol,
                double slack, double alpha, int l5, int n5, int* l, int* n, int* used) {
  float x[kMlpIn];
  mlp_features(op, norms, t, p, tol, x);
  float y[kMlpOut];
  mlp_predict_host(w, x, y);
  if (!std::isfinite(y[0]) || !std::isfinite(y[1])) {
    *used = 3;
    return false;
  }
  const int lp = std::min(60, std::max(0, (int)std::lround(y[0] * 8.0f)));
  const int mp = std::max(1, (int)std::lround(y[1] * 16.0f));
  // the judge: nodes the bound needs at this scaling (within the slack)
  const int nreq = quadnodes(std::min(tol * slack, 0.1), p, std::ldexp(alpha, -lp), 1.0, PHIQ_RULE_GAUSS);
  if (nreq < 0) {
    *used = 3;
    return false;
  }
  int m = mp;
  *used = 1;
  if (m < nreq + 1) {
    m = nreq + 1;
    *used = 2;
  }
  // a choice far costlier than Algorithm setup_quadrature's under the paper's
  // own count (m + l p chains) is rejected
  if ((double)(m + lp * p) > 1.5 * (double)((n5 + 1) + l5 * p)) {
    *used = 3;
    return false;
  }
  *l = lp;
  *n = m - 1;
  return true;
}

bool mlp_choose_empirical(const float* w, const phiq_kron_op* op, const double* norms, double t, int p,
                          double tol, double alpha, int l5, int n5, int* l, int* n, int* used) {
  *used = 0;
  if (tol < kEmpiricalTolMin) return false;
  float x[kMlpIn];
  mlp_features(op, norms, t, p, tol, x);
  float y[kMlpOut];
  mlp_predict_host(w, x, y);
  if (!std::isfinite(y[0]) || !std::isfinite(y[1])) {
    *used = 3;
    return false;
  }
  const int lp = std::min(60, std::max(0, (int)std::lround(y[0] * 8.0f)));
  // the norm at which the bound covers the measured errors, as a fraction
  // 10^y1 of ||tA||: never above the norm itself, never below a tenth of it
  const double ratio = std::pow(10.0, std::min(0.0, std::max(-1.0, (double)y[1])));
  const int nq = quadnodes(tol, p, std::ldexp(alpha * ratio, -lp), 1.0, PHIQ_RULE_GAUSS);
  if (nq < 0) {
    *used = 3;
    return false;
  }
  if ((double)(nq + 1 + lp * p) > 1.5 * (double)((n5 + 1) + l5 * p)) {
    *used = 3;
    return false;
  }
  *l = lp;
  *n = nq;
  *used = 4;
  return true;
}

namespace {

struct MlpBufs {
  void* mem = nullptr;
  float *H1, *H2, *Y, *dY, *dZ1, *dZ2;
  double *part, *loss_part;
  int chunks, nblk;
  ~MlpBufs() {
    if (mem) {
      (void)hipDeviceSynchronize();
      (void)hipFree(mem);
    }
  }
  phiq_status alloc(int B, int loss_rows) {
    chunks = std::max(1, std::min(64, B / 64));
    nblk = (B + 255) / 256;
    const size_t f = (size_t)B * (2 * kMlpHidden + kMlpOut) * 2;  // H1 H2 Y, dZ1 dZ2 dY
    const size_t bytes = f * sizeof(float) + ((size_t)chunks * kMlpParams + (size_t)loss_rows * nblk) * sizeof(double) + 1024;
    if (hipMalloc(&mem, bytes) != hipSuccess) {
      mem = nullptr;
      (void)hipGetLastError();
      return PHIQ_ERR_OOM;
    }
    float* q = (float*)mem;
    H1 = q; q += (size_t)B * kMlpHidden;
    H2 = q; q += (size_t)B * kMlpHidden;
    dZ1 = q; q += (size_t)B * kMlpHidden;
    dZ2 = q; q += (size_t)B * kMlpHidden;
    Y = q; q += (size_t)B * kMlpOut;
    dY = q; q += (size_t)B * kMlpOut;
    double* d = (double*)(((uintptr_t)q + 255) & ~(uintptr_t)255);
    part = d; d += (size_t)chunks * kMlpParams;
    loss_part = d;
    return PHIQ_OK;
  }
};

phiq_status grad_pass(MlpBufs& b, int B, const float* X, const float* T, const float* w, float* grad,
                      double* loss_part, hipStream_t st) {
  PHIQ_HIP(launch_mlp_forward(w, X, B, b.H1, b.H2, b.Y, st));
  PHIQ_HIP(launch_mlp_backward(w, T, b.H1, b.H2, b.Y, B, b.dY, b.dZ2, b.dZ1, loss_part, st));
  PHIQ_HIP(launch_mlp_wgrad(X, b.H1, b.H2, b.dZ1, b.dZ2, b.dY, B, b.chunks, b.part, grad, st));
  return PHIQ_OK;
}

}  // namespace
}  // namespace phiq

using namespace phiq;

extern "C" phiq_status phiq_mlp_forward(phiq_handle h, int B, const float* X, const float* w, float* Y,
                                        hipStream_t stream) {
  if (!h || B < 0 || (B > 0 && (!X || !w || !Y))) return PHIQ_ERR_INVALID_ARG;
  if (B == 0) return PHIQ_OK;
  PHIQ_HIP(launch_mlp_forward(w, X, B, nullptr, nullptr, Y, stream));
  return PHIQ_OK;
}

extern "C" phiq_status phiq_mlp_grad(phiq_handle h, int B, const float* X, const float* T, const float* w,
                                     float* grad, double* loss, hipStream_t stream) {
  if (!h || B < 1 || !X || !T || !w || !grad) return PHIQ_ERR_INVALID_ARG;
  MlpBufs b;
  PHIQ_TRY(b.alloc(B, 1));
  PHIQ_TRY(grad_pass(b, B, X, T, w, grad, b.loss_part, stream));
  if (loss) {
    std::vector<double> lp(b.nblk);
    PHIQ_HIP(hipMemcpyAsync(lp.data(), b.loss_part, sizeof(double) * b.nblk, hipMemcpyDeviceToHost, stream));
    PHIQ_HIP(hipStreamSynchronize(stream));
    double s = 0.0;
    for (double v : lp) s += v;
    *loss = s / ((double)B * kMlpOut);
  }
  PHIQ_HIP(hipStreamSynchronize(stream));
  return PHIQ_OK;
}

extern "C" phiq_status phiq_mlp_train(phiq_handle h, int B, const float* X, const float* T, float* w, int steps,
                                      float lr, float* loss_history) {
  if (!h || B < 1 || !X || !T || !w || steps < 0 || !(lr > 0) || !std::isfinite(lr)) return PHIQ_ERR_INVALID_ARG;
  MlpBufs b;
  PHIQ_TRY(b.alloc(B, std::max(1, steps)));
  float* dev = nullptr;
  const size_t nf = (size_t)B * (kMlpIn + kMlpOut) + 4 * (size_t)kMlpParams;
  if (hipMalloc((void**)&dev, nf * sizeof(float)) != hipSuccess) {
    (void)hipGetLastError();
    return PHIQ_ERR_OOM;
  }
  struct Free {
    float* p;
    ~Free() {
      (void)hipDeviceSynchronize();
      (void)hipFree(p);
    }
  } fr{dev};
  float* dX = dev;
  float* dT = dX + (size_t)B * kMlpIn;
  float* dw = dT + (size_t)B * kMlpOut;
  float* g = dw + kMlpParams;
  float* m = g + kMlpParams;
  float* v = m + kMlpParams;
  hipStream_t st = nullptr;
  PHIQ_HIP(hipStreamCreateWithFlags(&st, hipStreamNonBlocking));
  struct Stream {
    hipStream_t s;
    ~Stream() { (void)hipStreamDestroy(s); }
  } sg{st};
  PHIQ_HIP(hipMemcpyAsync(dX, X, sizeof(float) * B * kMlpIn, hipMemcpyHostToDevice, st));
  PHIQ_HIP(hipMemcpyAsync(dT, T, sizeof(float) * B * kMlpOut, hipMemcpyHostToDevice, st));
  PHIQ_HIP(hipMemcpyAsync(dw, w, sizeof(float) * kMlpParams, hipMemcpyHostToDevice, st));
  PHIQ_HIP(hipMemsetAsync(m, 0, sizeof(float) * 2 * kMlpParams, st));
  for (int s = 0; s < steps; ++s) {
    PHIQ_TRY(grad_pass(b, B, dX, dT, dw, g, b.loss_part + (size_t)s * b.nblk, st));
    PHIQ_HIP(launch_mlp_adam(dw, g, m, v, lr, 0.9f, 0.999f, 1e-8f, s + 1, st));
  }
  PHIQ_HIP(hipMemcpyAsync(w, dw, sizeof(float) * kMlpParams, hipMemcpyDeviceToHost, st));
  std::vector<double> lp((size_t)std::max(1, steps) * b.nblk);
  if (loss_history && steps > 0)
    PHIQ_HIP(hipMemcpyAsync(lp.data(), b.loss_part, sizeof(double) * lp.size(), hipMemcpyDeviceToHost, st));
  PHIQ_HIP(hipStreamSynchronize(st));
  if (loss_history)
    for (int s = 0; s < steps; ++s) {
      double sum = 0.0;
      for (int k = 0; k < b.nblk; ++k) sum += lp[(size_t)s * b.nblk + k];
      loss_history[s] = (float)(sum / ((double)B * kMlpOut));
    }
  return PHIQ_OK;
}
