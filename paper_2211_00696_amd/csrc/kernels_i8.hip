// Mode products on int8 slices (gfx950, v_mfma_i32_32x32x32_i8): an
// error-free split of the FP64 operands into S signed 7-bit digits
// (Ozaki-style splitting), the digit products exact in int32, the
// combination in FP64.
//
// Representation.  A vector x with exponent a (|x| < 2^a, up to a factor
// 1.9) is stored as S digit planes:
//   x = 2^a sum_{s=1}^{S} d_s 2^{-6-7(s-1)},  |d_s| <= 64 (<= 127 with the slack),
// d_1 = rint(64 x 2^-a), then each residual, scaled by 128, rounded again;
// every step is exact in FP64, so the truncation error is at most
// 2^{a-7S}.  The 1D factors carry one exponent per row; a tensor carries
// one exponent for all of it.
//
// Product.  out[i][j] = sum_k E[i][k] X[j][k] (the rotated mode product of
// the FP64 kernels) with E row i = 2^{e_i} sum_s e_s 2^{..}, X = 2^{x} sum_t
// x_t 2^{..}:  out = 2^{e_i + x - 12} sum_{g} 2^{-7g} sum_{s+t=g} P_st, P_st the
// exact int32 products of the digit planes; pairs with s + t > S are dropped
// (each is below 2^{-7S} of the scale).  One int32 accumulator per g.
//
// Layout.  A wave computes a 32 x 32 output tile: its 32 rows of E stay in
// registers for the whole launch (each lane holds half of one row: K/2
// digits per slice), the 32 columns of X are staged through LDS and shared by
// the block's waves (one wave per 32 rows of E, M = 32..128).  The lane
// holding row r, half g feeds k = g K/2 + 16 q + [0, 16) into MFMA step q,
// for A and B alike (the instruction sums over its 32 k in any order).
// Epilogues: digits of the output with the exponent x + delta, where 2^delta
// bounds ||E||_inf (the output stays below 2^{x + delta}); FP64 store; or the
// modified squaring combination.
#include <hip/hip_ext.h>
#include <hip/hip_runtime.h>

#include "phiq_internal.h"

// Launch with the profiler's start/stop events when they are armed
// (g_launch_events); `first` / `last` say which of the two this launch takes.
#define PHIQ_I8_LAUNCH(FIRST, LAST, K, G, B, SH, ST, ...)                                           \
  do {                                                                                             \
    if (g_launch_events[0])                                                                        \
      hipExtLaunchKernelGGL(K, G, B, SH, ST, (FIRST) ? (hipEvent_t)g_launch_events[0] : nullptr,    \
                            (LAST) ? (hipEvent_t)g_launch_events[1] : nullptr, 0, __VA_ARGS__);     \
    else                                                                                           \
      hipLaunchKernelGGL(K, G, B, SH, ST, __VA_ARGS__);                                            \
  } while (0)

namespace phiq {
namespace {

typedef int v4i __attribute__((ext_vector_type(4)));
typedef int v16i __attribute__((ext_vector_type(16)));

// S digits of y = 64 x 2^{-a} (|y| <= 121), written with stride ps
__device__ __forceinline__ void put_digits(double y, int S, int8_t* __restrict__ p, long long ps) {
  for (int s = 0; s < S; ++s) {
    const double d = rint(y);
    p[s * ps] = (int8_t)(int)d;
    y = (y - d) * 128.0;
  }
}

// Rows of length K (contiguous): one exponent per row, digits into planes
// [S][rows][K].  One wave per row.
__global__ void i8_slice_rows_kernel(const double* __restrict__ X, long long rows, int K, int S,
                                     int8_t* __restrict__ planes, int* __restrict__ ex) {
  const int lane = threadIdx.x & 63;
  const long long nw = ((long long)gridDim.x * blockDim.x) >> 6;
  const long long ps = rows * K;
  for (long long r = ((long long)blockIdx.x * blockDim.x + threadIdx.x) >> 6; r < rows; r += nw) {
    const double* x = X + r * K;
    double m = 0.0;
    for (int k = lane; k < K; k += 64) m = fmax(m, fabs(x[k]));
    for (int o = 32; o > 0; o >>= 1) m = fmax(m, __shfl_xor(m, o));
    const int a = (m > 0.0) ? ilogb(m) + 1 : 0;
    if (lane == 0) ex[r] = a;
    for (int k = lane; k < K; k += 64) put_digits(ldexp(x[k], 6 - a), S, planes + r * K + k, ps);
  }
}

// Partial max |x| of nt tensors (tensor r at X + r xs, N values): grid
// (nbx, nt), partial[r nbx + blockIdx.x].
__global__ void i8_absmax_kernel(const double* __restrict__ X, long long xs, long long N,
                                 double* __restrict__ partial) {
  __shared__ double red[4];
  const double* x = X + blockIdx.y * xs;
  double m = 0.0;
  for (long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x; i < N; i += (long long)gridDim.x * blockDim.x)
    m = fmax(m, fabs(x[i]));
  for (int o = 32; o > 0; o >>= 1) m = fmax(m, __shfl_xor(m, o));
  if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = m;
  __syncthreads();
  if (threadIdx.x == 0) {
    for (int w = 1; w < (int)(blockDim.x >> 6); ++w) m = fmax(m, red[w]);
    partial[blockIdx.y * gridDim.x + blockIdx.x] = m;
  }
}

// Tensor r: exponent from the nbx partial maxima (every block reduces them
// itself), digits into planes + r bstride (slice s at + s N), ex[r].
__global__ void i8_slice_tensor_kernel(const double* __restrict__ X, long long xs, long long N,
                                       const double* __restrict__ partial, int nbx, int S,
                                       int8_t* __restrict__ planes, long long bstride, int* __restrict__ ex) {
  __shared__ double red[4];
  const double* pr = partial + (long long)blockIdx.y * nbx;
  double m = 0.0;
  for (int i = threadIdx.x; i < nbx; i += blockDim.x) m = fmax(m, pr[i]);
  for (int o = 32; o > 0; o >>= 1) m = fmax(m, __shfl_xor(m, o));
  if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = m;
  __syncthreads();
  m = red[0];
  for (int w = 1; w < (int)(blockDim.x >> 6); ++w) m = fmax(m, red[w]);
  const int a = (m > 0.0) ? ilogb(m) + 1 : 0;
  if (blockIdx.x == 0 && threadIdx.x == 0) ex[blockIdx.y] = a;
  const double* x = X + blockIdx.y * xs;
  int8_t* p = planes + blockIdx.y * bstride;
  for (long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x; i < N; i += (long long)gridDim.x * blockDim.x)
    put_digits(ldexp(x[i], 6 - a), S, p + i, N);
}

// one wave per SIMD: the factor rows, the accumulators, the prefetched X
// digits and the digit epilogue take up to 512 registers
template <int S, int KQ, int MODE>
__global__ __launch_bounds__(256, 1) void i8_product_kernel(I8Args a) {
  constexpr int K = 32 * KQ;
  constexpr int ROW = K + 16;  // LDS row stride (bytes): spreads the 32 rows over the banks
  constexpr int HALF = K / 2;
  __shared__ __attribute__((aligned(16))) int8_t lds[S * 32 * ROW];
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6, g = lane >> 5, r = lane & 31;
  const int b = blockIdx.y;
  const bool active = 32 * w < a.M;
  const int i0 = 32 * w;
  const long long L = a.L;

  // this wave's rows of E for the whole launch
  v4i Ereg[S][KQ];
  {
    const int row = active ? i0 + r : 0;
    const int8_t* e = a.E + b * a.es + (long long)row * K + g * HALF;
#pragma unroll
    for (int s = 0; s < S; ++s)
#pragma unroll
      for (int q = 0; q < KQ; ++q) Ereg[s][q] = *(const v4i*)(e + s * a.esp + 16 * q);
  }
  const int ax = a.xe[b * a.xes];
  // exponents of the 16 output rows this lane holds (fixed for the launch)
  int erow[16];
#pragma unroll
  for (int e = 0; e < 16; ++e) erow[e] = active ? a.ee[b * a.ees + i0 + 8 * (e >> 2) + 4 * g + (e & 3)] : 0;
  const int8_t* X = a.X + b * a.xs;
  const int ntile = (int)(L / 32);
  constexpr int CHUNKS = S * 32 * K / 16;  // 16-byte pieces of one X tile
  constexpr int PER = (CHUNKS + 255) / 256;
  // the next tile's digits travel into registers while this tile is computed
  v4i pf[PER];
  auto fetch = [&](long long j0) {
#pragma unroll
    for (int u = 0; u < PER; ++u) {
      const int c = threadIdx.x + 256 * u;
      if (c < CHUNKS) {
        const int s = c / (32 * K / 16);
        const int rem = c - s * (32 * K / 16);
        const int row = rem / (K / 16), c16 = rem - row * (K / 16);
        pf[u] = *(const v4i*)(X + s * a.xsp + (j0 + row) * K + 16 * c16);
      }
    }
  };
  int js = blockIdx.x;
  if (js < ntile) fetch((long long)js * 32);
  for (; js < ntile; js += gridDim.x) {
    const long long j0 = (long long)js * 32;
    __syncthreads();  // the previous tile's reads are done
#pragma unroll
    for (int u = 0; u < PER; ++u) {
      const int c = threadIdx.x + 256 * u;
      if (c < CHUNKS) {
        const int s = c / (32 * K / 16);
        const int rem = c - s * (32 * K / 16);
        const int row = rem / (K / 16), c16 = rem - row * (K / 16);
        *(v4i*)(lds + s * 32 * ROW + row * ROW + 16 * c16) = pf[u];
      }
    }
    __syncthreads();
    if (js + (int)gridDim.x < ntile) fetch((long long)(js + gridDim.x) * 32);
    if (!active) continue;
    v16i acc[S];
#pragma unroll
    for (int q = 0; q < S; ++q) acc[q] = v16i{};
#pragma unroll
    for (int q = 0; q < KQ; ++q) {
      v4i B[S];
#pragma unroll
      for (int t = 0; t < S; ++t) B[t] = *(const v4i*)(lds + t * 32 * ROW + r * ROW + g * HALF + 16 * q);
#pragma unroll
      for (int s = 0; s < S; ++s)
#pragma unroll
        for (int t = 0; s + t < S; ++t)
          acc[s + t] = __builtin_amdgcn_mfma_i32_32x32x32_i8(Ereg[s][q], B[t], acc[s + t], 0, 0, 0);
    }
    const long long col = j0 + r;
#pragma unroll
    for (int e = 0; e < 16; ++e) {
      const int row = i0 + 8 * (e >> 2) + 4 * g + (e & 3);
      double v = 0.0;
#pragma unroll
      for (int q = S - 1; q >= 0; --q) v = v * (1.0 / 128.0) + (double)acc[q][e];
      const long long idx = (long long)row * L + col;
      const int sc = erow[e] + ax - 12;
      if (MODE == kI8Slice) {
        // digits of out 2^{-(ax + delta)} scaled by 64
        put_digits(ldexp(v, sc - ax - a.delta + 6), S, a.O8 + b * a.os8 + idx, a.osp8);
      } else if (MODE == kI8Store) {
        a.O[b * a.os + idx] = ldexp(v, sc);
      } else {  // modified squaring, order b + 1
        const int order = b + 1;
        double s = ldexp(v, sc);
        for (int jj = 1; jj <= order; ++jj) s += a.Yprev[(jj - 1) * a.yps + idx] * a.ifact[order - jj];
        a.O[b * a.os + idx] = ldexp(s, -order);
      }
    }
  }
  if (MODE == kI8Slice && blockIdx.x == 0 && threadIdx.x == 0) a.oe[b] = ax + a.delta;
}

template <int S, int KQ>
int launch_kq(const I8Args& a, int mode, dim3 grid, hipStream_t st) {
  if (mode == kI8Slice)
    PHIQ_I8_LAUNCH(true, true, (i8_product_kernel<S, KQ, kI8Slice>), grid, dim3(256), 0, st, a);
  else if (mode == kI8Store)
    PHIQ_I8_LAUNCH(true, true, (i8_product_kernel<S, KQ, kI8Store>), grid, dim3(256), 0, st, a);
  else
    PHIQ_I8_LAUNCH(true, true, (i8_product_kernel<S, KQ, kI8Square>), grid, dim3(256), 0, st, a);
  return hipGetLastError();
}

template <int S>
int launch_s(const I8Args& a, int mode, dim3 grid, hipStream_t st) {
  switch (a.K / 32) {
    case 1: return launch_kq<S, 1>(a, mode, grid, st);
    case 2: return launch_kq<S, 2>(a, mode, grid, st);
    case 3: return launch_kq<S, 3>(a, mode, grid, st);
    case 4: return launch_kq<S, 4>(a, mode, grid, st);
  }
  return hipErrorInvalidValue;
}

inline int grid_for(long long n) {
  const long long b = (n + 255) / 256;
  return (int)(b < 4096 ? (b > 0 ? b : 1) : 4096);
}

}  // namespace

int launch_i8_slice_rows(const double* X, long long rows, int K, int S, int8_t* planes, int* ex, void* stream) {
  if (rows <= 0) return hipSuccess;
  const long long blocks = (rows + 3) / 4;
  PHIQ_I8_LAUNCH(true, true, i8_slice_rows_kernel, dim3((unsigned)(blocks < 4096 ? blocks : 4096)), dim3(256), 0,
                 (hipStream_t)stream, X, rows, K, S, planes, ex);
  return hipGetLastError();
}

int launch_i8_slice_tensors(const double* X, long long xs, long long N, int nt, int S, double* partial, int nbx,
                            int8_t* planes, long long bstride, int* ex, void* stream) {
  if (nt <= 0 || N <= 0 || nbx < 1) return hipErrorInvalidValue;
  PHIQ_I8_LAUNCH(true, false, i8_absmax_kernel, dim3(nbx, nt), dim3(256), 0, (hipStream_t)stream, X, xs, N, partial);
  const int gx = grid_for(N) < 1024 ? grid_for(N) : 1024;
  PHIQ_I8_LAUNCH(false, true, i8_slice_tensor_kernel, dim3(gx, nt), dim3(256), 0, (hipStream_t)stream, X, xs, N,
                 partial, nbx, S, planes, bstride, ex);
  return hipGetLastError();
}

int launch_i8_product(const I8Args& a, int mode, void* stream) {
  if (a.M < 32 || a.M > 128 || a.M % 32 || a.K != a.M || a.L % 32 || a.nbatch < 1) return hipErrorInvalidValue;
  const long long ntile = a.L / 32;
  // about three blocks per CU over the batch; each keeps its factor rows for its tiles
  long long gx = (768 + a.nbatch - 1) / a.nbatch;
  if (gx > ntile) gx = ntile;
  if (gx < 1) gx = 1;
  const dim3 grid((unsigned)gx, (unsigned)a.nbatch);
  hipStream_t st = (hipStream_t)stream;
  switch (a.S) {
    case 5: return launch_s<5>(a, mode, grid, st);
    case 6: return launch_s<6>(a, mode, grid, st);
    case 7: return launch_s<7>(a, mode, grid, st);
  }
  return hipErrorInvalidValue;
}

}  // namespace phiq
