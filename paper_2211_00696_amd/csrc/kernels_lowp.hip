// Lower-precision mode products for gfx950: FP32 MFMA (v_mfma_f32_16x16x4_f32)
// and split bf16 with three products (v_mfma_f32_16x16x32_bf16), both with
// FP32 accumulation.  The 1D exponentials arrive already converted (FP32, or
// bf16 hi/lo pairs, made once per plan by convert_kernel); the tensor
// operand arrives as FP64 (input vector, squaring iterates) or FP32
// (intermediates between mode products) and is rounded while it is staged
// into LDS.  Node sums and the squaring combination in the epilogues are FP64.
//
// Split bf16: x = hi + lo with hi = bf16(x), lo = bf16(x - hi); a product
// a b is formed as hi_a hi_b + hi_a lo_b + lo_a hi_b (the dropped lo_a lo_b
// term is about 2^-16 of the product).
//
// Lane layouts (one wave, 64 lanes):
//   f32 16x16x4 : A lane l holds A[l%16][l/16], B lane l holds B[l/16][l%16]
//   bf16 16x16x32: A lane l holds A[l%16][8(l/16) .. 8(l/16)+7], B likewise
//   D (4 floats) : lane l, element e holds D[4(l/16) + e][l%16]
#include <hip/hip_ext.h>
#include <hip/hip_runtime.h>

#include "phiq_internal.h"

namespace phiq {

// Launch, with the live-timing events attached when they are set.
#define PHIQ_LAUNCH(K, G, B, SH, ST, ...)                                                                 \
  do {                                                                                                    \
    if (g_launch_events[0])                                                                               \
      hipExtLaunchKernelGGL(K, G, B, SH, ST, (hipEvent_t)g_launch_events[0], (hipEvent_t)g_launch_events[1], \
                            0, __VA_ARGS__);                                                              \
    else                                                                                                  \
      hipLaunchKernelGGL(K, G, B, SH, ST, __VA_ARGS__);                                                   \
  } while (0)


typedef float f4 __attribute__((ext_vector_type(4)));
typedef __bf16 bf8 __attribute__((ext_vector_type(8)));
typedef double dv2 __attribute__((ext_vector_type(2)));

enum { LP_F32 = 0, LP_BF16X3 = 1 };

// ---------------------------------------------------------------------------
// one-off conversion of the 1D exponentials
// ---------------------------------------------------------------------------
__global__ void convert_kernel(const double* __restrict__ src, long long count, int mode, void* a, void* b,
                               const int* __restrict__ stop) {
  if (stop && *stop) return;
  for (long long i = blockIdx.x * (long long)blockDim.x + threadIdx.x; i < count; i += (long long)gridDim.x * blockDim.x) {
    const double x = src[i];
    if (mode == LP_F32) {
      ((float*)a)[i] = (float)x;
    } else {
      const __bf16 hi = (__bf16)(float)x;
      ((__bf16*)a)[i] = hi;
      ((__bf16*)b)[i] = (__bf16)(float)(x - (double)(float)hi);
    }
  }
}

int launch_convert(const double* src, long long count, phiq_precision prec, void* a, void* b, void* stream,
                   const int* stop) {
  if (count <= 0) return hipSuccess;
  const int mode = prec == PHIQ_PREC_FP32 ? LP_F32 : LP_BF16X3;
  const long long nb = std::min<long long>(4096, (count + 255) / 256);
  PHIQ_LAUNCH(convert_kernel, dim3((unsigned)nb), dim3(256), 0, (hipStream_t)stream, src, count, mode, a, b, stop);
  return hipGetLastError();
}

// ---------------------------------------------------------------------------
// tiles
// ---------------------------------------------------------------------------
template <int MODE, int BM_>
struct Lp {
  static constexpr int BM = BM_, BN = 64;
  static constexpr int BK = (MODE == LP_F32) ? 16 : 32;
  static constexpr int WAVES_M = 2, WAVES_N = 2, NT = 256;
  static constexpr int WM = BM / WAVES_M, WN = BN / WAVES_N;
  static constexpr int TM = WM / 16, TN = WN / 16;
  // padded rows keep 16-byte alignment and spread the MFMA reads over banks
  static constexpr int LDK = (MODE == LP_F32) ? BK + 4 : BK + 8;
  // elements per thread and chunk
  static constexpr int A_PER = BM * BK / NT, B_PER = BN * BK / NT;
  static_assert(A_PER * NT == BM * BK && B_PER * NT == BN * BK, "tile");
  static_assert(A_PER % 4 == 0 && B_PER % 4 == 0, "vector staging");
};

template <int MODE, int BM>
struct LpStage;
template <int BM>
struct alignas(16) LpStage<LP_F32, BM> {
  using C = Lp<LP_F32, BM>;
  float A[C::BM * C::LDK];
  float B[C::BN * C::LDK];
};
template <int BM>
struct alignas(16) LpStage<LP_BF16X3, BM> {
  using C = Lp<LP_BF16X3, BM>;
  __bf16 Ahi[C::BM * C::LDK];
  __bf16 Alo[C::BM * C::LDK];
  __bf16 Bhi[C::BN * C::LDK];
  __bf16 Blo[C::BN * C::LDK];
};

// Registers of one prefetched chunk.  Each thread owns PER consecutive k
// of one row (PER = 8 or 16 elements).
template <int MODE, int BM, class TIn>
struct LpRegs {
  using C = Lp<MODE, BM>;
  // A operand (already converted): FP32 -> floats; BF16 -> hi and lo bf16
  typename std::conditional<MODE == LP_F32, float, __bf16>::type a0[C::A_PER], a1[MODE == LP_F32 ? 1 : C::A_PER];
  TIn b[C::B_PER];
};

// Clamped, branch-free loads; the k tail is zeroed when the A operand is
// written to LDS (rows past the end only feed outputs that are not stored).
template <int MODE, int BM, class TIn, bool VEC>
__device__ __forceinline__ void lp_load(const void* __restrict__ Ea, const void* __restrict__ Eb,
                                        const TIn* __restrict__ X, int M, int K, int L, int m0, int n0, int k0,
                                        LpRegs<MODE, BM, TIn>& r) {
  using C = Lp<MODE, BM>;
  // A: thread t covers row t / (BK/A_PER), k offset (t % (BK/A_PER)) * A_PER
  {
    constexpr int TPR = C::BK / C::A_PER;
    const int row = m0 + threadIdx.x / TPR, kk = (threadIdx.x % TPR) * C::A_PER;
    const int rc = row < M ? row : M - 1;
    if constexpr (MODE == LP_F32) {
      const float* g = (const float*)Ea + (long long)rc * K;
#pragma unroll
      for (int i = 0; i < C::A_PER; i += 4) {
        const int k = k0 + kk + i;
        if constexpr (VEC) {
          const f4 v = *(const f4*)(g + (k < K ? k : 0));
          r.a0[i] = v.x; r.a0[i + 1] = v.y; r.a0[i + 2] = v.z; r.a0[i + 3] = v.w;
        } else {
#pragma unroll
          for (int j = 0; j < 4; ++j) r.a0[i + j] = g[(k + j) < K ? k + j : 0];
        }
      }
    } else {
      const __bf16* gh = (const __bf16*)Ea + (long long)rc * K;
      const __bf16* gl = (const __bf16*)Eb + (long long)rc * K;
#pragma unroll
      for (int i = 0; i < C::A_PER; i += 8) {
        const int k = k0 + kk + i;
        if constexpr (VEC) {
          const bf8 h = *(const bf8*)(gh + (k < K ? k : 0));
          const bf8 l = *(const bf8*)(gl + (k < K ? k : 0));
#pragma unroll
          for (int j = 0; j < 8; ++j) {
            r.a0[i + j] = h[j];
            r.a1[i + j] = l[j];
          }
        } else {
#pragma unroll
          for (int j = 0; j < 8; ++j) {
            const int kj = (k + j) < K ? k + j : 0;
            r.a0[i + j] = gh[kj];
            r.a1[i + j] = gl[kj];
          }
        }
      }
    }
  }
  // B: thread t covers row t / (BK/B_PER), k offset (t % (BK/B_PER)) * B_PER
  {
    constexpr int TPR = C::BK / C::B_PER;
    const int row = n0 + threadIdx.x / TPR, kk = (threadIdx.x % TPR) * C::B_PER;
    const int rc = row < L ? row : L - 1;
    const TIn* g = X + (long long)rc * K;
    constexpr int W = 16 / sizeof(TIn);  // elements per 16-byte load
#pragma unroll
    for (int i = 0; i < C::B_PER; i += W) {
      const int k = k0 + kk + i;
      if constexpr (VEC) {
        if constexpr (sizeof(TIn) == 4) {
          const f4 v = *(const f4*)(g + (k < K ? k : 0));
          r.b[i] = v.x; r.b[i + 1] = v.y; r.b[i + 2] = v.z; r.b[i + 3] = v.w;
        } else {
          const dv2 v = *(const dv2*)(g + (k < K ? k : 0));
          r.b[i] = v.x; r.b[i + 1] = v.y;
        }
      } else {
#pragma unroll
        for (int j = 0; j < W; ++j) r.b[i + j] = g[(k + j) < K ? k + j : 0];
      }
    }
  }
}

template <int MODE, int BM, class TIn>
__device__ __forceinline__ void lp_store(LpStage<MODE, BM>& s, const LpRegs<MODE, BM, TIn>& r, int k0, int K) {
  using C = Lp<MODE, BM>;
  {
    constexpr int TPR = C::BK / C::A_PER;
    const int row = threadIdx.x / TPR, kk = (threadIdx.x % TPR) * C::A_PER;
    if constexpr (MODE == LP_F32) {
#pragma unroll
      for (int i = 0; i < C::A_PER; i += 4) {
        f4 v;
#pragma unroll
        for (int j = 0; j < 4; ++j) v[j] = (k0 + kk + i + j < K) ? r.a0[i + j] : 0.f;
        *(f4*)&s.A[row * C::LDK + kk + i] = v;
      }
    } else {
#pragma unroll
      for (int i = 0; i < C::A_PER; i += 8) {
        bf8 h, l;
#pragma unroll
        for (int j = 0; j < 8; ++j) {
          const bool ok = k0 + kk + i + j < K;
          h[j] = ok ? r.a0[i + j] : (__bf16)0.f;
          l[j] = ok ? r.a1[i + j] : (__bf16)0.f;
        }
        *(bf8*)&s.Ahi[row * C::LDK + kk + i] = h;
        *(bf8*)&s.Alo[row * C::LDK + kk + i] = l;
      }
    }
  }
  {
    constexpr int TPR = C::BK / C::B_PER;
    const int row = threadIdx.x / TPR, kk = (threadIdx.x % TPR) * C::B_PER;
    if constexpr (MODE == LP_F32) {
#pragma unroll
      for (int i = 0; i < C::B_PER; i += 4) {
        f4 v;
#pragma unroll
        for (int j = 0; j < 4; ++j) v[j] = (float)r.b[i + j];
        *(f4*)&s.B[row * C::LDK + kk + i] = v;
      }
    } else {
#pragma unroll
      for (int i = 0; i < C::B_PER; i += 8) {
        bf8 h, l;
#pragma unroll
        for (int j = 0; j < 8; ++j) {
          const float x = (float)r.b[i + j];
          const __bf16 hb = (__bf16)x;
          h[j] = hb;
          l[j] = (__bf16)(sizeof(TIn) == 8 ? (float)((double)r.b[i + j] - (double)(float)hb) : x - (float)hb);
        }
        *(bf8*)&s.Bhi[row * C::LDK + kk + i] = h;
        *(bf8*)&s.Blo[row * C::LDK + kk + i] = l;
      }
    }
  }
}

template <int MODE, int BM>
__device__ __forceinline__ void lp_mma(const LpStage<MODE, BM>& sm, f4 (&acc)[Lp<MODE, BM>::TM][Lp<MODE, BM>::TN]) {
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

// acc = E[m0:m0+BM, :] X[n0:n0+BN, :]^T, double-buffered LDS, prefetch two
// chunks ahead, one barrier per chunk
template <int MODE, int BM, class TIn, bool VEC>
__device__ __forceinline__ void lp_tile(const void* Ea, const void* Eb, const TIn* __restrict__ X, int M, int K,
                                        int L, int m0, int n0, LpStage<MODE, BM> (&sm)[2],
                                        f4 (&acc)[Lp<MODE, BM>::TM][Lp<MODE, BM>::TN]) {
  using C = Lp<MODE, BM>;
#pragma unroll
  for (int i = 0; i < C::TM; ++i)
#pragma unroll
    for (int j = 0; j < C::TN; ++j) acc[i][j] = (f4){0.f, 0.f, 0.f, 0.f};
  LpRegs<MODE, BM, TIn> r;
  const int nch = (K + C::BK - 1) / C::BK;
  lp_load<MODE, BM, TIn, VEC>(Ea, Eb, X, M, K, L, m0, n0, 0, r);
  lp_store<MODE, BM, TIn>(sm[0], r, 0, K);
  if (nch > 1) lp_load<MODE, BM, TIn, VEC>(Ea, Eb, X, M, K, L, m0, n0, C::BK, r);
  __syncthreads();
  for (int c = 0; c < nch; ++c) {
    if (c + 1 < nch) {
      lp_store<MODE, BM, TIn>(sm[(c + 1) & 1], r, (c + 1) * C::BK, K);
      if (c + 2 < nch) lp_load<MODE, BM, TIn, VEC>(Ea, Eb, X, M, K, L, m0, n0, (c + 2) * C::BK, r);
    }
    lp_mma<MODE, BM>(sm[c & 1], acc);
    __syncthreads();
  }
}

constexpr int kXcdsLp = 8;

template <class C>
__device__ __forceinline__ bool lp_tile_of_block(int M, int L, int nb, int& m0, int& n0, int& b) {
  const int mtiles = (M + C::BM - 1) / C::BM;
  const long long T = (long long)mtiles * ((L + C::BN - 1) / C::BN) * nb;
  const long long per = (T + kXcdsLp - 1) / kXcdsLp;
  const long long t = (long long)(blockIdx.x % kXcdsLp) * per + blockIdx.x / kXcdsLp;
  if (t >= T) return false;
  m0 = (int)(t % mtiles) * C::BM;
  const long long r = t / mtiles;
  b = (int)(r % nb);
  n0 = (int)(r / nb) * C::BN;
  return true;
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

template <int MODE>
__device__ __forceinline__ const void* e_ptr(const TtmArgs& a, const void* base, int b) {
  const size_t esz = (MODE == LP_F32) ? sizeof(float) : sizeof(__bf16);
  return (const char*)base + (size_t)b * a.es * esz;
}

template <int MODE, int BM, class TIn, class TOut, bool VEC>
__global__ __launch_bounds__(256) void ttm_lp_store_kernel(TtmArgs a) {
  using C = Lp<MODE, BM>;
  __shared__ LpStage<MODE, BM> sm[2];
  if (a.stop && *a.stop) return;
  int m0, n0, b;
  if (!lp_tile_of_block<C>(a.M, a.L, a.nbatch, m0, n0, b)) return;
  f4 acc[C::TM][C::TN];
  lp_tile<MODE, BM, TIn, VEC>(e_ptr<MODE>(a, a.Ea, b), e_ptr<MODE>(a, a.Eb, b), (const TIn*)a.X + b * a.xs, a.M, a.K,
                              a.L, m0, n0, sm, acc);
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

template <int MODE, int BM, class TIn, int NP, bool VEC>
__global__ __launch_bounds__(256) void ttm_lp_accum_kernel(TtmArgs a) {
  using C = Lp<MODE, BM>;
  __shared__ LpStage<MODE, BM> sm[2];
  int m0, n0, bb;
  if (!lp_tile_of_block<C>(a.M, a.L, 1, m0, n0, bb)) return;
  double y[NP][C::TM][C::TN][4];
#pragma unroll
  for (int q = 0; q < NP; ++q)
#pragma unroll
    for (int i = 0; i < C::TM; ++i)
#pragma unroll
      for (int j = 0; j < C::TN; ++j)
#pragma unroll
        for (int e = 0; e < 4; ++e) y[q][i][j][e] = 0.0;
  for (int b = 0; b < a.nbatch; ++b) {
    f4 acc[C::TM][C::TN];
    lp_tile<MODE, BM, TIn, VEC>(e_ptr<MODE>(a, a.Ea, b), e_ptr<MODE>(a, a.Eb, b), (const TIn*)a.X + b * a.xs, a.M,
                                a.K, a.L, m0, n0, sm, acc);
#pragma unroll
    for (int q = 0; q < NP; ++q) {
      const double w = ldexp(a.coef[q * a.ldcoef + b], a.cexp);
#pragma unroll
      for (int i = 0; i < C::TM; ++i)
#pragma unroll
        for (int j = 0; j < C::TN; ++j)
#pragma unroll
          for (int e = 0; e < 4; ++e) y[q][i][j][e] += w * (double)acc[i][j][e];
    }
  }
#pragma unroll
  for (int q = 0; q < NP; ++q) {
    double* Y = a.Y + q * a.ys;
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
            Y[idx] = a.yacc ? Y[idx] + y[q][i][j][e] : y[q][i][j][e];
          }
        }
      }
  }
}

template <int MODE, int BM, class TIn, bool VEC>
__global__ __launch_bounds__(256) void ttm_lp_square_kernel(TtmArgs a) {
  using C = Lp<MODE, BM>;
  __shared__ LpStage<MODE, BM> sm[2];
  int m0, n0, b;
  if (!lp_tile_of_block<C>(a.M, a.L, a.nbatch, m0, n0, b)) return;
  f4 acc[C::TM][C::TN];
  lp_tile<MODE, BM, TIn, VEC>(e_ptr<MODE>(a, a.Ea, b), e_ptr<MODE>(a, a.Eb, b), (const TIn*)a.X + b * a.xs, a.M, a.K,
                              a.L, m0, n0, sm, acc);
  const int order = b + 1 + a.order0;
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
          for (int jj = 1; jj <= order; ++jj) s += a.Yprev[(jj - 1) * a.yps + idx] * a.ifact[order - jj];
          O[idx] = a.yacc ? O[idx] + scale * s : scale * s;
        }
      }
    }
}

// All p orders of one squaring step per block (p <= 4), each y_j tile read
// once and kept in registers.
template <int MODE, int BM, class TIn, int NP, bool VEC>
__global__ __launch_bounds__(256) void ttm_lp_square_all_kernel(TtmArgs a) {
  using C = Lp<MODE, BM>;
  __shared__ LpStage<MODE, BM> sm[2];
  int m0, n0, bb;
  if (!lp_tile_of_block<C>(a.M, a.L, 1, m0, n0, bb)) return;
  double ys[NP][C::TM][C::TN][4];
#pragma unroll
  for (int i = 0; i < NP; ++i) {
#pragma unroll
    for (int ti = 0; ti < C::TM; ++ti)
#pragma unroll
      for (int tj = 0; tj < C::TN; ++tj) {
        const int col = n0 + lp_col<C>(tj);
#pragma unroll
        for (int e = 0; e < 4; ++e) {
          const int row = m0 + lp_row<C>(ti, e);
          const int rc = row < a.M ? row : a.M - 1, cc = col < a.L ? col : a.L - 1;
          ys[i][ti][tj][e] = a.Yprev[i * a.yps + (long long)rc * a.L + cc];
        }
      }
    f4 acc[C::TM][C::TN];
    lp_tile<MODE, BM, TIn, VEC>(a.Ea, a.Eb, (const TIn*)a.X + i * a.xs, a.M, a.K, a.L, m0, n0, sm, acc);
    const double scale = ldexp(1.0, -(i + 1));
    double* O = (double*)a.O + i * a.os;
#pragma unroll
    for (int ti = 0; ti < C::TM; ++ti)
#pragma unroll
      for (int tj = 0; tj < C::TN; ++tj) {
        const int col = n0 + lp_col<C>(tj);
#pragma unroll
        for (int e = 0; e < 4; ++e) {
          const int row = m0 + lp_row<C>(ti, e);
          double s = (double)acc[ti][tj][e];
#pragma unroll
          for (int j = 0; j <= i; ++j) s += ys[j][ti][tj][e] * a.ifact[i - j];
          if (row < a.M && col < a.L) O[(long long)row * a.L + col] = scale * s;
        }
      }
  }
}

namespace {
inline unsigned cdivu(long long a, long long b) { return (unsigned)((a + b - 1) / b); }

template <int MODE, int BM>
dim3 lp_grid(const TtmArgs& a, int nb) {
  using C = Lp<MODE, BM>;
  const long long T = (long long)cdivu(a.M, C::BM) * cdivu(a.L, C::BN) * nb;
  return dim3((unsigned)(((T + kXcdsLp - 1) / kXcdsLp) * kXcdsLp), 1, 1);
}

// vector staging: rows of 8 elements stay 16-byte aligned
bool lp_vec(const TtmArgs& a) {
  return (a.K % 8 == 0) && (((uintptr_t)a.Ea | (uintptr_t)a.Eb | (uintptr_t)a.X) % 16 == 0) && (a.es % 8 == 0) &&
         (a.xs % 8 == 0);
}

template <int MODE, int BM, class TIn, class TOut>
int store_go(const TtmArgs& a, hipStream_t st) {
  const dim3 g = lp_grid<MODE, BM>(a, a.nbatch);
  if (lp_vec(a))
    PHIQ_LAUNCH((ttm_lp_store_kernel<MODE, BM, TIn, TOut, true>), g, dim3(256), 0, st, a);
  else
    PHIQ_LAUNCH((ttm_lp_store_kernel<MODE, BM, TIn, TOut, false>), g, dim3(256), 0, st, a);
  return hipGetLastError();
}

template <int MODE, int BM>
int store_dispatch(const TtmArgs& a, hipStream_t st) {
  if (a.x_f32 && a.o_f32) return store_go<MODE, BM, float, float>(a, st);
  if (a.x_f32) return store_go<MODE, BM, float, double>(a, st);
  if (a.o_f32) return store_go<MODE, BM, double, float>(a, st);
  return store_go<MODE, BM, double, double>(a, st);
}

template <int MODE>
int store_mode(const TtmArgs& a, hipStream_t st) {
  return a.M > 64 ? store_dispatch<MODE, 128>(a, st) : store_dispatch<MODE, 64>(a, st);
}

template <int MODE, class TIn, bool VEC>
int accum_go(const TtmArgs& a, hipStream_t st) {
  const dim3 g = lp_grid<MODE, 64>(a, 1);
  switch (a.np) {
    case 1: PHIQ_LAUNCH((ttm_lp_accum_kernel<MODE, 64, TIn, 1, VEC>), g, dim3(256), 0, st, a); break;
    case 2: PHIQ_LAUNCH((ttm_lp_accum_kernel<MODE, 64, TIn, 2, VEC>), g, dim3(256), 0, st, a); break;
    case 3: PHIQ_LAUNCH((ttm_lp_accum_kernel<MODE, 64, TIn, 3, VEC>), g, dim3(256), 0, st, a); break;
    default: PHIQ_LAUNCH((ttm_lp_accum_kernel<MODE, 64, TIn, 4, VEC>), g, dim3(256), 0, st, a); break;
  }
  return hipGetLastError();
}

template <int MODE>
int accum_mode(const TtmArgs& a, hipStream_t st) {
  const bool v = lp_vec(a);
  if (a.x_f32) return v ? accum_go<MODE, float, true>(a, st) : accum_go<MODE, float, false>(a, st);
  return v ? accum_go<MODE, double, true>(a, st) : accum_go<MODE, double, false>(a, st);
}

template <int MODE, int BM, class TIn>
int square_go(const TtmArgs& a, hipStream_t st) {
  const dim3 g = lp_grid<MODE, BM>(a, a.nbatch);
  if (lp_vec(a))
    PHIQ_LAUNCH((ttm_lp_square_kernel<MODE, BM, TIn, true>), g, dim3(256), 0, st, a);
  else
    PHIQ_LAUNCH((ttm_lp_square_kernel<MODE, BM, TIn, false>), g, dim3(256), 0, st, a);
  return hipGetLastError();
}

template <int MODE, class TIn, bool VEC>
int square_all_go(const TtmArgs& a, hipStream_t st) {
  const dim3 g = lp_grid<MODE, 64>(a, 1);
  switch (a.nbatch) {
    case 1: PHIQ_LAUNCH((ttm_lp_square_all_kernel<MODE, 64, TIn, 1, VEC>), g, dim3(256), 0, st, a); break;
    case 2: PHIQ_LAUNCH((ttm_lp_square_all_kernel<MODE, 64, TIn, 2, VEC>), g, dim3(256), 0, st, a); break;
    case 3: PHIQ_LAUNCH((ttm_lp_square_all_kernel<MODE, 64, TIn, 3, VEC>), g, dim3(256), 0, st, a); break;
    default: PHIQ_LAUNCH((ttm_lp_square_all_kernel<MODE, 64, TIn, 4, VEC>), g, dim3(256), 0, st, a); break;
  }
  return hipGetLastError();
}

template <int MODE>
int square_mode(const TtmArgs& a, hipStream_t st) {
  // an order offset or an accumulating store needs the per-order kernel
  if (a.nbatch <= 4 && a.es == 0 && a.order0 == 0 && !a.yacc) {
    const bool v = lp_vec(a);
    if (a.x_f32) return v ? square_all_go<MODE, float, true>(a, st) : square_all_go<MODE, float, false>(a, st);
    return v ? square_all_go<MODE, double, true>(a, st) : square_all_go<MODE, double, false>(a, st);
  }
  if (a.M > 64) return a.x_f32 ? square_go<MODE, 128, float>(a, st) : square_go<MODE, 128, double>(a, st);
  return a.x_f32 ? square_go<MODE, 64, float>(a, st) : square_go<MODE, 64, double>(a, st);
}
}  // namespace

int launch_ttm_store_lowp(const TtmArgs& a, phiq_precision prec, void* stream) {
  hipStream_t st = (hipStream_t)stream;
  if (!a.Ea || (prec == PHIQ_PREC_BF16X3 && !a.Eb)) return hipErrorInvalidValue;
  if (prec == PHIQ_PREC_FP32) return store_mode<LP_F32>(a, st);
  if (prec == PHIQ_PREC_BF16X3) return store_mode<LP_BF16X3>(a, st);
  return hipErrorInvalidValue;
}

int launch_ttm_accum_lowp(const TtmArgs& a, phiq_precision prec, void* stream) {
  hipStream_t st = (hipStream_t)stream;
  if (!a.Ea || (prec == PHIQ_PREC_BF16X3 && !a.Eb)) return hipErrorInvalidValue;
  if (prec == PHIQ_PREC_FP32) return accum_mode<LP_F32>(a, st);
  if (prec == PHIQ_PREC_BF16X3) return accum_mode<LP_BF16X3>(a, st);
  return hipErrorInvalidValue;
}

int launch_ttm_square_lowp(const TtmArgs& a, phiq_precision prec, void* stream) {
  hipStream_t st = (hipStream_t)stream;
  if (!a.Ea || (prec == PHIQ_PREC_BF16X3 && !a.Eb)) return hipErrorInvalidValue;
  if (prec == PHIQ_PREC_FP32) return square_mode<LP_F32>(a, st);
  if (prec == PHIQ_PREC_BF16X3) return square_mode<LP_BF16X3>(a, st);
  return hipErrorInvalidValue;
}

}  // namespace phiq
