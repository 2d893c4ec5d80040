// Elementwise parts of the ETD-RK4 step (Cox-Matthews) for
// u' = -A u + F(u), F(u) = c1 u + c3 u^3 (gfx950).  Each kernel reads and
// writes every element once (HBM-bound); grid-stride loops.
#include <hip/hip_runtime.h>

#include "phiq_internal.h"

namespace phiq {
namespace {

__device__ __forceinline__ double cubic(double x, double c1, double c3) { return x * (c1 + c3 * x * x); }

__global__ void etd_nonlin_kernel(const double* __restrict__ x, double* __restrict__ fx, long long n, double c1,
                                  double c3) {
  for (long long i = blockIdx.x * (long long)blockDim.x + threadIdx.x; i < n; i += (long long)gridDim.x * blockDim.x)
    fx[i] = cubic(x[i], c1, c3);
}

__global__ void etd_stage_kernel(const double* __restrict__ x, const double* __restrict__ y, double s,
                                 double* __restrict__ a, double* __restrict__ fa, long long n, double c1, double c3) {
  for (long long i = blockIdx.x * (long long)blockDim.x + threadIdx.x; i < n; i += (long long)gridDim.x * blockDim.x) {
    const double v = x[i] + s * y[i];
    if (a) a[i] = v;
    fa[i] = cubic(v, c1, c3);
  }
}

__global__ void etd_stage_b_kernel(const double* __restrict__ x, const double* __restrict__ y, double s,
                                   const double* __restrict__ fu, const double* __restrict__ fa,
                                   double* __restrict__ mix, double* __restrict__ sum, long long n, double c1,
                                   double c3) {
  for (long long i = blockIdx.x * (long long)blockDim.x + threadIdx.x; i < n; i += (long long)gridDim.x * blockDim.x) {
    const double fb = cubic(x[i] + s * y[i], c1, c3);
    mix[i] = 2.0 * fb - fu[i];
    sum[i] = fa[i] + fb;
  }
}

// Cox-Matthews update with f1 = phi1 - 3 phi2 + 4 phi3, f2 = phi2 - 2 phi3,
// f3 = -phi2 + 4 phi3 applied to F(u), F(a) + F(b) and F(c).
__global__ void etd_final_kernel(const double* __restrict__ e, const double* __restrict__ g, double h,
                                 double* __restrict__ u, long long n) {
  for (long long i = blockIdx.x * (long long)blockDim.x + threadIdx.x; i < n; i += (long long)gridDim.x * blockDim.x) {
    const double* g1 = g + i;
    const double* g2 = g + 4 * n + i;
    const double* g3 = g + 8 * n + i;
    const double f1 = g1[n] - 3.0 * g1[2 * n] + 4.0 * g1[3 * n];
    const double f2 = g2[2 * n] - 2.0 * g2[3 * n];
    const double f3 = -g3[2 * n] + 4.0 * g3[3 * n];
    u[i] = e[i] + h * (f1 + 2.0 * f2 + f3);
  }
}

// Linear-combination form: the vectors b_j that enter sum_j phi_j b_j.
// fx = F(x), s = hs fx (the stage's phi_1 vector at h/2)
__global__ void etd_cf_stage_kernel(const double* __restrict__ x, double* __restrict__ fx, double* __restrict__ s,
                                    double hs, long long n, double c1, double c3) {
  for (long long i = blockIdx.x * (long long)blockDim.x + threadIdx.x; i < n; i += (long long)gridDim.x * blockDim.x) {
    const double f = cubic(x[i], c1, c3);
    fx[i] = f;
    s[i] = hs * f;
  }
}

// F(b): s = hs (2 F(b) - F(u)), fab = F(a) + F(b)
__global__ void etd_cf_b_kernel(const double* __restrict__ b, const double* __restrict__ fu,
                                const double* __restrict__ fa, double* __restrict__ s, double* __restrict__ fab,
                                double hs, long long n, double c1, double c3) {
  for (long long i = blockIdx.x * (long long)blockDim.x + threadIdx.x; i < n; i += (long long)gridDim.x * blockDim.x) {
    const double fb = cubic(b[i], c1, c3);
    s[i] = hs * (2.0 * fb - fu[i]);
    fab[i] = fa[i] + fb;
  }
}

// The final update h [f1 F(u) + 2 f2 (F(a) + F(b)) + f3 F(c)] regrouped by
// phi_j: b_1 = h F(u), b_2 = h (-3 F(u) + 2 (F(a)+F(b)) - F(c)),
// b_3 = 4 h (F(u) - (F(a)+F(b)) + F(c)).
__global__ void etd_cf_final_kernel(const double* __restrict__ c, const double* __restrict__ fu,
                                    const double* __restrict__ fab, double* __restrict__ b1, double* __restrict__ b2,
                                    double* __restrict__ b3, double h, long long n, double c1, double c3) {
  for (long long i = blockIdx.x * (long long)blockDim.x + threadIdx.x; i < n; i += (long long)gridDim.x * blockDim.x) {
    const double fc = cubic(c[i], c1, c3);
    const double f0 = fu[i], f2 = fab[i];
    b1[i] = h * f0;
    b2[i] = h * (-3.0 * f0 + 2.0 * f2 - fc);
    b3[i] = 4.0 * h * (f0 - f2 + fc);
  }
}

__global__ void etd_copy_kernel(const double* __restrict__ x, double* __restrict__ y, long long n) {
  for (long long i = blockIdx.x * (long long)blockDim.x + threadIdx.x; i < n; i += (long long)gridDim.x * blockDim.x)
    y[i] = x[i];
}

inline int grid_for(long long n) {
  const long long b = (n + 255) / 256;
  return (int)(b < 2048 ? (b > 0 ? b : 1) : 2048);
}

}  // namespace

int launch_etd_nonlin(const double* x, double* fx, long long n, double c1, double c3, void* stream) {
  hipLaunchKernelGGL(etd_nonlin_kernel, dim3(grid_for(n)), dim3(256), 0, (hipStream_t)stream, x, fx, n, c1, c3);
  return hipGetLastError();
}

int launch_etd_stage(const double* x, const double* y, double s, double* a, double* fa, long long n, double c1,
                     double c3, void* stream) {
  hipLaunchKernelGGL(etd_stage_kernel, dim3(grid_for(n)), dim3(256), 0, (hipStream_t)stream, x, y, s, a, fa, n, c1,
                     c3);
  return hipGetLastError();
}

int launch_etd_stage_b(const double* x, const double* y, double s, const double* fu, const double* fa, double* mix,
                       double* sum, long long n, double c1, double c3, void* stream) {
  hipLaunchKernelGGL(etd_stage_b_kernel, dim3(grid_for(n)), dim3(256), 0, (hipStream_t)stream, x, y, s, fu, fa, mix,
                     sum, n, c1, c3);
  return hipGetLastError();
}

int launch_etd_final(const double* e, const double* g, double h, double* u, long long n, void* stream) {
  hipLaunchKernelGGL(etd_final_kernel, dim3(grid_for(n)), dim3(256), 0, (hipStream_t)stream, e, g, h, u, n);
  return hipGetLastError();
}

int launch_etd_cf_stage(const double* x, double* fx, double* s, double hs, long long n, double c1, double c3,
                        void* stream) {
  hipLaunchKernelGGL(etd_cf_stage_kernel, dim3(grid_for(n)), dim3(256), 0, (hipStream_t)stream, x, fx, s, hs, n, c1,
                     c3);
  return hipGetLastError();
}

int launch_etd_cf_b(const double* b, const double* fu, const double* fa, double* s, double* fab, double hs,
                    long long n, double c1, double c3, void* stream) {
  hipLaunchKernelGGL(etd_cf_b_kernel, dim3(grid_for(n)), dim3(256), 0, (hipStream_t)stream, b, fu, fa, s, fab, hs, n,
                     c1, c3);
  return hipGetLastError();
}

int launch_etd_cf_final(const double* c, const double* fu, const double* fab, double* b1, double* b2, double* b3,
                        double h, long long n, double c1, double c3, void* stream) {
  hipLaunchKernelGGL(etd_cf_final_kernel, dim3(grid_for(n)), dim3(256), 0, (hipStream_t)stream, c, fu, fab, b1, b2,
                     b3, h, n, c1, c3);
  return hipGetLastError();
}

int launch_etd_copy(const double* x, double* y, long long n, void* stream) {
  hipLaunchKernelGGL(etd_copy_kernel, dim3(grid_for(n)), dim3(256), 0, (hipStream_t)stream, x, y, n);
  return hipGetLastError();
}

}  // namespace phiq
