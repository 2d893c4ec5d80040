// Lower-precision mode products for gfx950: FP32 MFMA (v_mfma_f32_16x16x4_f32)
// and split-bf16 with three products (v_mfma_f32_16x16x32_bf16), both with
// FP32 accumulation.  Operands arrive as FP64 (the 1D exponentials, the input
// vector, the squaring iterates) or FP32 (intermediate tensors) and are
// rounded while they are staged into LDS.  The node sums and the squaring
// combination in the epilogues are carried out in FP64.
//
// Split bf16: x = hi + lo with hi = bf16(x), lo = bf16(x - hi); a product
// a b is formed as hi_a hi_b + hi_a lo_b + lo_a hi_b (the lo_a lo_b term,
// about 2^-16 of the product, is dropped).
//
// Lane layouts (one wave, 64 lanes):
//   f32 16x16x4 : A lane l holds A[l%16][l/16], B lane l holds B[l/16][l%16]
//   bf16 16x16x32: A lane l holds A[l%16][8(l/16) .. 8(l/16)+7], B likewise
//                  with k = 8(l/16) + j and column l%16
//   D (4 floats) : lane l, element e holds D[4(l/16) + e][l%16]
#include <hip/hip_runtime.h>

#include "phiq_internal.h"

namespace phiq {

typedef float f4 __attribute__((ext_vector_type(4)));
typedef __bf16 bf8 __attribute__((ext_vector_type(8)));

enum { LP_F32 = 0, LP_BF16X3 = 1 };

template <int MODE, int BM_>
struct Lp {
  static constexpr int BM = BM_, BN = 64;
  static constexpr int BK = (MODE == LP_F32) ? 16 : 32;
  static constexpr int WAVES_M = 2, WAVES_N = 2, NT = 256;
  static constexpr int WM = BM / WAVES_M, WN = BN / WAVES_N;
  static constexpr int TM = WM / 16, TN = WN / 16;
  static constexpr int LDK = (MODE == LP_F32) ? BK + 1 : BK + 8;  // padded row, in elements
  static constexpr int A_PER = BM * BK / NT, B_PER = BN * BK / NT;
  static_assert(A_PER * NT == BM * BK && B_PER * NT == BN * BK, "tile");
};

template <class T>
__device__ __forceinline__ double ld_as_double(const T* p) {
  return (double)*p;
}

// LDS storage of one staged chunk
template <int MODE, int BM>
struct LpSmem;
template <int BM>
struct alignas(16) LpSmem<LP_F32, BM> {
  using C = Lp<LP_F32, BM>;
  float A[C::BM * C::LDK];
  float B[C::BN * C::LDK];
};
template <int BM>
struct alignas(16) LpSmem<LP_BF16X3, BM> {
  using C = Lp<LP_BF16X3, BM>;
  __bf16 Ahi[C::BM * C::LDK];
  __bf16 Alo[C::BM * C::LDK];
  __bf16 Bhi[C::BN * C::LDK];
  __bf16 Blo[C::BN * C::LDK];
};

template <int ROWS, int BK, int NT, int PER, class T>
__device__ __forceinline__ void lp_load(const T* __restrict__ g, long long ld, int r0, int rows_valid, int k0,
                                        int k_valid, double (&reg)[PER]) {
#pragma unroll
  for (int i = 0; i < PER; ++i) {
    const int e = threadIdx.x + i * NT;
    const int r = e / BK, kk = e % BK;
    const int row = r0 + r, k = k0 + kk;
    reg[i] = (row < rows_valid && k < k_valid) ? ld_as_double(g + (long long)row * ld + k) : 0.0;
  }
}

template <int BK, int NT, int PER, int LDK>
__device__ __forceinline__ void lp_store_f32(float* s, const double (&reg)[PER]) {
#pragma unroll
  for (int i = 0; i < PER; ++i) {
    const int e = threadIdx.x + i * NT;
    s[(e / BK) * LDK + (e % BK)] = (float)reg[i];
  }
}

template <int BK, int NT, int PER, int LDK>
__device__ __forceinline__ void lp_store_split(__bf16* shi, __bf16* slo, const double (&reg)[PER]) {
#pragma unroll
  for (int i = 0; i < PER; ++i) {
    const int e = threadIdx.x + i * NT;
    const double x = reg[i];
    const __bf16 hi = (__bf16)(float)x;
    const __bf16 lo = (__bf16)(float)(x - (double)(float)hi);
    const int o = (e / BK) * LDK + (e % BK);
    shi[o] = hi;
    slo[o] = lo;
  }
}

template <int MODE, int BM>
__device__ __forceinline__ void lp_stage(LpSmem<MODE, BM>& sm, const double (&ra)[Lp<MODE, BM>::A_PER],
                                         const double (&rb)[Lp<MODE, BM>::B_PER]) {
  using C = Lp<MODE, BM>;
  if constexpr (MODE == LP_F32) {
    lp_store_f32<C::BK, C::NT, C::A_PER, C::LDK>(sm.A, ra);
    lp_store_f32<C::BK, C::NT, C::B_PER, C::LDK>(sm.B, rb);
  } else {
    lp_store_split<C::BK, C::NT, C::A_PER, C::LDK>(sm.Ahi, sm.Alo, ra);
    lp_store_split<C::BK, C::NT, C::B_PER, C::LDK>(sm.Bhi, sm.Blo, rb);
  }
}

template <int MODE, int BM>
__device__ __forceinline__ void lp_mma(const LpSmem<MODE, BM>& sm, f4 (&acc)[Lp<MODE, BM>::TM][Lp<MODE, BM>::TN]) {
  using C = Lp<MODE, BM>;
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int wm = wave / C::WAVES_N, wn = wave % C::WAVES_N;
  const int ra = wm * C::WM + (lane & 15), rb = wn * C::WN + (lane & 15);
  if constexpr (MODE == LP_F32) {
#pragma unroll
    for (int k4 = 0; k4 < C::BK / 4; ++k4) {
      float a[C::TM], b[C::TN];
#pragma unroll
      for (int i = 0; i < C::TM; ++i) a[i] = sm.A[(ra + 16 * i) * C::LDK + 4 * k4 + (lane >> 4)];
#pragma unroll
      for (int j = 0; j < C::TN; ++j) b[j] = sm.B[(rb + 16 * j) * C::LDK + 4 * k4 + (lane >> 4)];
#pragma unroll
      for (int i = 0; i < C::TM; ++i)
#pragma unroll
        for (int j = 0; j < C::TN; ++j) acc[i][j] = __builtin_amdgcn_mfma_f32_16x16x4f32(a[i], b[j], acc[i][j], 0, 0, 0);
    }
  } else {
    const int ko = 8 * (lane >> 4);
    bf8 ah[C::TM], al[C::TM], bh[C::TN], bl[C::TN];
#pragma unroll
    for (int i = 0; i < C::TM; ++i) {
      ah[i] = *(const bf8*)&sm.Ahi[(ra + 16 * i) * C::LDK + ko];
      al[i] = *(const bf8*)&sm.Alo[(ra + 16 * i) * C::LDK + ko];
    }
#pragma unroll
    for (int j = 0; j < C::TN; ++j) {
      bh[j] = *(const bf8*)&sm.Bhi[(rb + 16 * j) * C::LDK + ko];
      bl[j] = *(const bf8*)&sm.Blo[(rb + 16 * j) * C::LDK + ko];
    }
#pragma unroll
    for (int i = 0; i < C::TM; ++i)
#pragma unroll
      for (int j = 0; j < C::TN; ++j) {
        acc[i][j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(al[i], bh[j], acc[i][j], 0, 0, 0);
        acc[i][j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(ah[i], bl[j], acc[i][j], 0, 0, 0);
        acc[i][j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(ah[i], bh[j], acc[i][j], 0, 0, 0);
      }
  }
}

// acc = E[m0:m0+BM, :] X[n0:n0+BN, :]^T in FP32 accumulation
template <int MODE, int BM, class TIn>
__device__ __forceinline__ void lp_tile(const double* __restrict__ E, const TIn* __restrict__ X, int M, int K, int L,
                                        int m0, int n0, LpSmem<MODE, BM>& sm,
                                        f4 (&acc)[Lp<MODE, BM>::TM][Lp<MODE, BM>::TN]) {
  using C = Lp<MODE, BM>;
#pragma unroll
  for (int i = 0; i < C::TM; ++i)
#pragma unroll
    for (int j = 0; j < C::TN; ++j) acc[i][j] = (f4){0.f, 0.f, 0.f, 0.f};
  double ra[C::A_PER], rb[C::B_PER];
  lp_load<C::BM, C::BK, C::NT, C::A_PER>(E, K, m0, M, 0, K, ra);
  lp_load<C::BN, C::BK, C::NT, C::B_PER>(X, K, n0, L, 0, K, rb);
  for (int k0 = 0; k0 < K; k0 += C::BK) {
    __syncthreads();
    lp_stage<MODE, BM>(sm, ra, rb);
    __syncthreads();
    if (k0 + C::BK < K) {
      lp_load<C::BM, C::BK, C::NT, C::A_PER>(E, K, m0, M, k0 + C::BK, K, ra);
      lp_load<C::BN, C::BK, C::NT, C::B_PER>(X, K, n0, L, k0 + C::BK, K, rb);
    }
    lp_mma<MODE, BM>(sm, acc);
  }
}

template <class C>
__device__ __forceinline__ void lp_origin(int M, int& m0, int& n0) {
  const int mtiles = (M + C::BM - 1) / C::BM;
  m0 = (blockIdx.x % mtiles) * C::BM;
  n0 = (blockIdx.x / mtiles) * C::BN;
}
template <class C>
__device__ __forceinline__ int lp_row(int i, int e) {
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  return (wave / C::WAVES_N) * C::WM + 16 * i + 4 * (lane >> 4) + e;
}
template <class C>
__device__ __forceinline__ int lp_col(int j) {
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  return (wave % C::WAVES_N) * C::WN + 16 * j + (lane & 15);
}

template <int MODE, int BM, class TIn, class TOut>
__global__ __launch_bounds__(256) void ttm_lp_store_kernel(TtmArgs a) {
  using C = Lp<MODE, BM>;
  __shared__ LpSmem<MODE, BM> sm;
  int m0, n0;
  lp_origin<C>(a.M, m0, n0);
  const int b = blockIdx.y;
  f4 acc[C::TM][C::TN];
  lp_tile<MODE, BM, TIn>(a.E + b * a.es, (const TIn*)a.X + b * a.xs, a.M, a.K, a.L, m0, n0, sm, acc);
  TOut* O = (TOut*)a.O + b * a.os;
#pragma unroll
  for (int i = 0; i < C::TM; ++i)
#pragma unroll
    for (int j = 0; j < C::TN; ++j) {
      const int col = n0 + lp_col<C>(j);
#pragma unroll
      for (int e = 0; e < 4; ++e) {
        const int row = m0 + lp_row<C>(i, e);
        if (row < a.M && col < a.L) O[(long long)row * a.L + col] = (TOut)acc[i][j][e];
      }
    }
}

// node sums in FP64 over all nodes of the batch (np <= 4)
template <int MODE, int BM, class TIn>
__global__ __launch_bounds__(256) void ttm_lp_accum_kernel(TtmArgs a) {
  using C = Lp<MODE, BM>;
  __shared__ LpSmem<MODE, BM> sm;
  int m0, n0;
  lp_origin<C>(a.M, m0, n0);
  double y[4][C::TM][C::TN][4];
#pragma unroll
  for (int q = 0; q < 4; ++q)
#pragma unroll
    for (int i = 0; i < C::TM; ++i)
#pragma unroll
      for (int j = 0; j < C::TN; ++j)
#pragma unroll
        for (int e = 0; e < 4; ++e) y[q][i][j][e] = 0.0;
  for (int b = 0; b < a.nbatch; ++b) {
    f4 acc[C::TM][C::TN];
    lp_tile<MODE, BM, TIn>(a.E + b * a.es, (const TIn*)a.X + b * a.xs, a.M, a.K, a.L, m0, n0, sm, acc);
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      if (q < a.np) {
        const double w = a.coef[q * a.ldcoef + b];
#pragma unroll
        for (int i = 0; i < C::TM; ++i)
#pragma unroll
          for (int j = 0; j < C::TN; ++j)
#pragma unroll
            for (int e = 0; e < 4; ++e) y[q][i][j][e] += w * (double)acc[i][j][e];
      }
    }
  }
#pragma unroll
  for (int q = 0; q < 4; ++q) {
    if (q < a.np) {
      double* Y = a.Y + q * a.ys;
#pragma unroll
      for (int i = 0; i < C::TM; ++i)
#pragma unroll
        for (int j = 0; j < C::TN; ++j) {
          const int col = n0 + lp_col<C>(j);
#pragma unroll
          for (int e = 0; e < 4; ++e) {
            const int row = m0 + lp_row<C>(i, e);
            if (row < a.M && col < a.L) Y[(long long)row * a.L + col] = y[q][i][j][e];
          }
        }
    }
  }
}

// modified squaring combination in FP64 (eq. squaring)
template <int MODE, int BM, class TIn>
__global__ __launch_bounds__(256) void ttm_lp_square_kernel(TtmArgs a) {
  using C = Lp<MODE, BM>;
  __shared__ LpSmem<MODE, BM> sm;
  int m0, n0;
  lp_origin<C>(a.M, m0, n0);
  const int b = blockIdx.y;
  f4 acc[C::TM][C::TN];
  lp_tile<MODE, BM, TIn>(a.E + b * a.es, (const TIn*)a.X + b * a.xs, a.M, a.K, a.L, m0, n0, sm, acc);
  const int order = b + 1;
  const double scale = ldexp(1.0, -order);
  double* O = (double*)a.O + b * a.os;
#pragma unroll
  for (int i = 0; i < C::TM; ++i)
#pragma unroll
    for (int j = 0; j < C::TN; ++j) {
      const int col = n0 + lp_col<C>(j);
#pragma unroll
      for (int e = 0; e < 4; ++e) {
        const int row = m0 + lp_row<C>(i, e);
        if (row < a.M && col < a.L) {
          const long long idx = (long long)row * a.L + col;
          double s = (double)acc[i][j][e];
          double inv_fact = 1.0;
          for (int jj = order; jj >= 1; --jj) {
            s += a.Yprev[(jj - 1) * a.yps + idx] * inv_fact;
            inv_fact /= (double)(order - jj + 1);
          }
          O[idx] = scale * s;
        }
      }
    }
}

namespace {
inline unsigned cdivu(long long a, long long b) { return (unsigned)((a + b - 1) / b); }

template <int MODE, int BM>
dim3 lp_grid(const TtmArgs& a, int nb) {
  using C = Lp<MODE, BM>;
  return dim3(cdivu(a.M, C::BM) * cdivu(a.L, C::BN), nb, 1);
}

template <int MODE, int BM>
int store_dispatch(const TtmArgs& a, hipStream_t st) {
  const dim3 g = lp_grid<MODE, BM>(a, a.nbatch);
  if (a.x_f32 && a.o_f32)
    hipLaunchKernelGGL((ttm_lp_store_kernel<MODE, BM, float, float>), g, dim3(256), 0, st, a);
  else if (a.x_f32)
    hipLaunchKernelGGL((ttm_lp_store_kernel<MODE, BM, float, double>), g, dim3(256), 0, st, a);
  else if (a.o_f32)
    hipLaunchKernelGGL((ttm_lp_store_kernel<MODE, BM, double, float>), g, dim3(256), 0, st, a);
  else
    hipLaunchKernelGGL((ttm_lp_store_kernel<MODE, BM, double, double>), g, dim3(256), 0, st, a);
  return hipGetLastError();
}

template <int MODE>
int store_mode(const TtmArgs& a, hipStream_t st) {
  return a.M > 64 ? store_dispatch<MODE, 128>(a, st) : store_dispatch<MODE, 64>(a, st);
}

template <int MODE>
int accum_mode(const TtmArgs& a, hipStream_t st) {
  const dim3 g = lp_grid<MODE, 64>(a, 1);
  if (a.x_f32)
    hipLaunchKernelGGL((ttm_lp_accum_kernel<MODE, 64, float>), g, dim3(256), 0, st, a);
  else
    hipLaunchKernelGGL((ttm_lp_accum_kernel<MODE, 64, double>), g, dim3(256), 0, st, a);
  return hipGetLastError();
}

template <int MODE, int BM>
int square_dispatch(const TtmArgs& a, hipStream_t st) {
  const dim3 g = lp_grid<MODE, BM>(a, a.nbatch);
  if (a.x_f32)
    hipLaunchKernelGGL((ttm_lp_square_kernel<MODE, BM, float>), g, dim3(256), 0, st, a);
  else
    hipLaunchKernelGGL((ttm_lp_square_kernel<MODE, BM, double>), g, dim3(256), 0, st, a);
  return hipGetLastError();
}

template <int MODE>
int square_mode(const TtmArgs& a, hipStream_t st) {
  return a.M > 64 ? square_dispatch<MODE, 128>(a, st) : square_dispatch<MODE, 64>(a, st);
}
}  // namespace

int launch_ttm_store_lowp(const TtmArgs& a, phiq_precision prec, void* stream) {
  hipStream_t st = (hipStream_t)stream;
  if (prec == PHIQ_PREC_FP32) return store_mode<LP_F32>(a, st);
  if (prec == PHIQ_PREC_BF16X3) return store_mode<LP_BF16X3>(a, st);
  return hipErrorInvalidValue;
}

int launch_ttm_accum_lowp(const TtmArgs& a, phiq_precision prec, void* stream) {
  hipStream_t st = (hipStream_t)stream;
  if (prec == PHIQ_PREC_FP32) return accum_mode<LP_F32>(a, st);
  if (prec == PHIQ_PREC_BF16X3) return accum_mode<LP_BF16X3>(a, st);
  return hipErrorInvalidValue;
}

int launch_ttm_square_lowp(const TtmArgs& a, phiq_precision prec, void* stream) {
  hipStream_t st = (hipStream_t)stream;
  if (prec == PHIQ_PREC_FP32) return square_mode<LP_F32>(a, st);
  if (prec == PHIQ_PREC_BF16X3) return square_mode<LP_BF16X3>(a, st);
  return hipErrorInvalidValue;
}

}  // namespace phiq
