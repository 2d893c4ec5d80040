// Elementwise parts of the exponential Runge-Kutta methods of Section 5 for
// Problem 3 (Hochbruck-Ostermann) on (0,1)^2: g(t, u) = 1/(1 + u^2) + f(x, y, t)
// with the manufactured source f that makes u = x(1-x) y(1-y) e^t the exact
// solution, f = u_ex + 2 e^t (x(1-x) + y(1-y)) - 1/(1 + u_ex^2).  Nodes
// x_i = (i+1)/(n+1), row-major (x slowest).  HBM-bound, grid-stride loops.
#include <hip/hip_runtime.h>

#include "phiq_internal.h"

namespace phiq {
namespace {

__device__ __forceinline__ double g_ho(double u, long long idx, int n, double t) {
  const double h = 1.0 / (double)(n + 1);
  const double x = (double)(idx / n + 1) * h, y = (double)(idx % n + 1) * h;
  const double qx = x * (1.0 - x), qy = y * (1.0 - y);
  const double et = exp(t);
  const double ue = qx * qy * et;
  return 1.0 / (1.0 + u * u) + ue + 2.0 * et * (qx + qy) - 1.0 / (1.0 + ue * ue);
}

// g = g(t, e + sa a + sb b) (b may be null); with copy != null also copy = e
__global__ void exprk_stage_kernel(const double* __restrict__ e, const double* __restrict__ a, double sa,
                                   const double* __restrict__ b, double sb, int n, double t,
                                   double* __restrict__ g, double* __restrict__ copy) {
  const long long N = (long long)n * n;
  for (long long i = blockIdx.x * (long long)blockDim.x + threadIdx.x; i < N; i += (long long)gridDim.x * blockDim.x) {
    double u = e[i];
    if (a) u += sa * a[i];
    if (b) u += sb * b[i];
    if (copy) copy[i] = e[i];
    g[i] = g_ho(u, i, n, t);
  }
}

// out = x + sa a + sb b (a, b may be null)
__global__ void exprk_comb_kernel(const double* x, const double* a, double sa, const double* b, double sb,
                                  double* out, long long N) {  // out may alias x or a
  for (long long i = blockIdx.x * (long long)blockDim.x + threadIdx.x; i < N; i += (long long)gridDim.x * blockDim.x) {
    double v = x[i];
    if (a) v += sa * a[i];
    if (b) v += sb * b[i];
    out[i] = v;
  }
}

// out = sa a + sb b (b may be null; out may alias a or b)
__global__ void exprk_axpby_kernel(const double* a, double sa, const double* b, double sb, double* out, long long N) {
  for (long long i = blockIdx.x * (long long)blockDim.x + threadIdx.x; i < N; i += (long long)gridDim.x * blockDim.x) {
    double v = sa * a[i];
    if (b) v += sb * b[i];
    out[i] = v;
  }
}

inline int grid_for(long long n) {
  const long long b = (n + 255) / 256;
  return (int)(b < 2048 ? (b > 0 ? b : 1) : 2048);
}

}  // namespace

int launch_exprk_stage(const double* e, const double* a, double sa, const double* b, double sb, int n, double t,
                       double* g, double* copy, void* stream) {
  const long long N = (long long)n * n;
  hipLaunchKernelGGL(exprk_stage_kernel, dim3(grid_for(N)), dim3(256), 0, (hipStream_t)stream, e, a, sa, b, sb, n, t,
                     g, copy);
  return hipGetLastError();
}

int launch_exprk_comb(const double* x, const double* a, double sa, const double* b, double sb, double* out,
                      long long N, void* stream) {
  hipLaunchKernelGGL(exprk_comb_kernel, dim3(grid_for(N)), dim3(256), 0, (hipStream_t)stream, x, a, sa, b, sb, out, N);
  return hipGetLastError();
}

int launch_exprk_axpby(const double* a, double sa, const double* b, double sb, double* out, long long N,
                       void* stream) {
  hipLaunchKernelGGL(exprk_axpby_kernel, dim3(grid_for(N)), dim3(256), 0, (hipStream_t)stream, a, sa, b, sb, out, N);
  return hipGetLastError();
}

}  // namespace phiq
