// HIP kernels for gfx950 (CDNA4): FP64 MFMA mode products with fused
// node-sum and squaring epilogues, small batched GEMMs and the truncated
// Taylor series used for the 1D exponentials.
//
// MFMA building block: v_mfma_f64_16x16x4_f64 (one wave, 64 lanes).
//   A operand: lane l holds A[l % 16][l / 16]      (16 x 4)
//   B operand: lane l holds B[l / 16][l % 16]      (4 x 16)
//   D (4 doubles): lane l, element e holds D[l / 16 + 4 e][l % 16]
#include <hip/hip_runtime.h>

#include "phiq_internal.h"

namespace phiq {

typedef double d4 __attribute__((ext_vector_type(4)));

template <int BM_, int BN_, int BK_, int WAVES_M_, int WAVES_N_>
struct Tile {
  static constexpr int BM = BM_, BN = BN_, BK = BK_;
  static constexpr int WAVES_M = WAVES_M_, WAVES_N = WAVES_N_;
  static constexpr int NT = 64 * WAVES_M_ * WAVES_N_;
  static constexpr int WM = BM_ / WAVES_M_, WN = BN_ / WAVES_N_;
  static constexpr int TM = WM / 16, TN = WN / 16;
  static constexpr int LDK = BK_ + 2;  // padded row length in LDS (doubles)
  static constexpr int A_PER = BM_ * BK_ / NT;
  static constexpr int B_PER = BN_ * BK_ / NT;
  static_assert(A_PER * NT == BM_ * BK_ && B_PER * NT == BN_ * BK_, "tile not divisible");
  static_assert(TM * 16 == WM && TN * 16 == WN && BK_ % 4 == 0, "wave tile");
};

using Tile64 = Tile<64, 64, 16, 2, 2>;
using Tile128 = Tile<128, 64, 16, 2, 2>;
using Tile256 = Tile<256, 64, 16, 4, 1>;
using Tile32 = Tile<32, 32, 16, 1, 1>;

// ---------------------------------------------------------------------------
// Staging: rows [r0, r0+ROWS) x k-chunk [k0, k0+BK) of a row-major matrix with
// row length ld (k contiguous), zero outside (rows_valid, k_valid).
// ---------------------------------------------------------------------------
template <int ROWS, int BK, int NT, int PER>
__device__ __forceinline__ void load_kmajor(const double* __restrict__ g, long long ld, int r0,
                                            int rows_valid, int k0, int k_valid, double (&reg)[PER]) {
#pragma unroll
  for (int i = 0; i < PER; ++i) {
    const int e = threadIdx.x + i * NT;
    const int r = e / BK, kk = e % BK;
    const int row = r0 + r, k = k0 + kk;
    reg[i] = (row < rows_valid && k < k_valid) ? g[(long long)row * ld + k] : 0.0;
  }
}
template <int BK, int NT, int PER, int LDK>
__device__ __forceinline__ void store_kmajor(double* s, const double (&reg)[PER]) {
#pragma unroll
  for (int i = 0; i < PER; ++i) {
    const int e = threadIdx.x + i * NT;
    s[(e / BK) * LDK + (e % BK)] = reg[i];
  }
}
// Rows of B are k (n contiguous in global): element (kk, c) of the chunk is
// B[(k0+kk) * ld + c0 + c]; stored transposed as s[c * LDK + kk].
template <int COLS, int BK, int NT, int PER>
__device__ __forceinline__ void load_nmajor(const double* __restrict__ g, long long ld, int c0,
                                            int cols_valid, int k0, int k_valid, double (&reg)[PER]) {
#pragma unroll
  for (int i = 0; i < PER; ++i) {
    const int e = threadIdx.x + i * NT;
    const int kk = e / COLS, c = e % COLS;
    const int k = k0 + kk, col = c0 + c;
    reg[i] = (col < cols_valid && k < k_valid) ? g[(long long)k * ld + col] : 0.0;
  }
}
template <int COLS, int NT, int PER, int LDK>
__device__ __forceinline__ void store_nmajor(double* s, const double (&reg)[PER]) {
#pragma unroll
  for (int i = 0; i < PER; ++i) {
    const int e = threadIdx.x + i * NT;
    s[(e % COLS) * LDK + (e / COLS)] = reg[i];
  }
}

template <class C>
__device__ __forceinline__ void zero_acc(d4 (&acc)[C::TM][C::TN]) {
#pragma unroll
  for (int i = 0; i < C::TM; ++i)
#pragma unroll
    for (int j = 0; j < C::TN; ++j) acc[i][j] = (d4){0.0, 0.0, 0.0, 0.0};
}

template <class C>
__device__ __forceinline__ void mma_chunk(const double* As, const double* Bs, d4 (&acc)[C::TM][C::TN]) {
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int wm = wave / C::WAVES_N, wn = wave % C::WAVES_N;
  const double* a_base = As + (wm * C::WM + (lane & 15)) * C::LDK + (lane >> 4);
  const double* b_base = Bs + (wn * C::WN + (lane & 15)) * C::LDK + (lane >> 4);
#pragma unroll
  for (int k4 = 0; k4 < C::BK / 4; ++k4) {
    double a[C::TM], b[C::TN];
#pragma unroll
    for (int i = 0; i < C::TM; ++i) a[i] = a_base[i * 16 * C::LDK + 4 * k4];
#pragma unroll
    for (int j = 0; j < C::TN; ++j) b[j] = b_base[j * 16 * C::LDK + 4 * k4];
#pragma unroll
    for (int i = 0; i < C::TM; ++i)
#pragma unroll
      for (int j = 0; j < C::TN; ++j) acc[i][j] = __builtin_amdgcn_mfma_f64_16x16x4f64(a[i], b[j], acc[i][j], 0, 0, 0);
  }
}

// acc += E[m0:m0+BM, :] * X[n0:n0+BN, :]^T  (E: M x K, X: L x K, both k-contiguous)
template <class C>
__device__ __forceinline__ void tile_nt(const double* __restrict__ E, const double* __restrict__ X, int M,
                                        int K, int L, int m0, int n0, double* As, double* Bs,
                                        d4 (&acc)[C::TM][C::TN]) {
  double ra[C::A_PER], rb[C::B_PER];
  load_kmajor<C::BM, C::BK, C::NT, C::A_PER>(E, K, m0, M, 0, K, ra);
  load_kmajor<C::BN, C::BK, C::NT, C::B_PER>(X, K, n0, L, 0, K, rb);
  for (int k0 = 0; k0 < K; k0 += C::BK) {
    __syncthreads();
    store_kmajor<C::BK, C::NT, C::A_PER, C::LDK>(As, ra);
    store_kmajor<C::BK, C::NT, C::B_PER, C::LDK>(Bs, rb);
    __syncthreads();
    if (k0 + C::BK < K) {
      load_kmajor<C::BM, C::BK, C::NT, C::A_PER>(E, K, m0, M, k0 + C::BK, K, ra);
      load_kmajor<C::BN, C::BK, C::NT, C::B_PER>(X, K, n0, L, k0 + C::BK, K, rb);
    }
    mma_chunk<C>(As, Bs, acc);
  }
}

// acc += A[m0:m0+BM, :] * B[:, n0:n0+BN]  (A: n x n, B: n x n, row-major)
template <class C>
__device__ __forceinline__ void tile_nn(const double* __restrict__ A, const double* __restrict__ B, int n,
                                        int m0, int n0, double* As, double* Bs, d4 (&acc)[C::TM][C::TN]) {
  double ra[C::A_PER], rb[C::B_PER];
  load_kmajor<C::BM, C::BK, C::NT, C::A_PER>(A, n, m0, n, 0, n, ra);
  load_nmajor<C::BN, C::BK, C::NT, C::B_PER>(B, n, n0, n, 0, n, rb);
  for (int k0 = 0; k0 < n; k0 += C::BK) {
    __syncthreads();
    store_kmajor<C::BK, C::NT, C::A_PER, C::LDK>(As, ra);
    store_nmajor<C::BN, C::NT, C::B_PER, C::LDK>(Bs, rb);
    __syncthreads();
    if (k0 + C::BK < n) {
      load_kmajor<C::BM, C::BK, C::NT, C::A_PER>(A, n, m0, n, k0 + C::BK, n, ra);
      load_nmajor<C::BN, C::BK, C::NT, C::B_PER>(B, n, n0, n, k0 + C::BK, n, rb);
    }
    mma_chunk<C>(As, Bs, acc);
  }
}

// Output coordinates of accumulator element (i, j, e) for this lane.
template <class C>
__device__ __forceinline__ int acc_row(int i, int e) {
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  return (wave / C::WAVES_N) * C::WM + 16 * i + (lane >> 4) + 4 * e;
}
template <class C>
__device__ __forceinline__ int acc_col(int j) {
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  return (wave % C::WAVES_N) * C::WN + 16 * j + (lane & 15);
}

// ---------------------------------------------------------------------------
// Mode products (rotated layout), three epilogues.
// grid: x = (L tile, M tile) with the M tile fastest, so the blocks that read
// the same X tile are adjacent; y = batch (store / square) or 1 (node sum)
// ---------------------------------------------------------------------------
template <class C>
__device__ __forceinline__ void tile_origin(int M, int& m0, int& n0) {
  const int mtiles = (M + C::BM - 1) / C::BM;
  m0 = (blockIdx.x % mtiles) * C::BM;
  n0 = (blockIdx.x / mtiles) * C::BN;
}

template <class C>
__global__ __launch_bounds__(C::NT) void ttm_store_kernel(TtmArgs a) {
  __shared__ double As[C::BM * C::LDK];
  __shared__ double Bs[C::BN * C::LDK];
  int m0, n0;
  tile_origin<C>(a.M, m0, n0);
  const int b = blockIdx.y;
  d4 acc[C::TM][C::TN];
  zero_acc<C>(acc);
  tile_nt<C>(a.E + b * a.es, (const double*)a.X + b * a.xs, a.M, a.K, a.L, m0, n0, As, Bs, acc);
  double* O = (double*)a.O + b * a.os;
#pragma unroll
  for (int i = 0; i < C::TM; ++i)
#pragma unroll
    for (int j = 0; j < C::TN; ++j) {
      const int col = n0 + acc_col<C>(j);
#pragma unroll
      for (int e = 0; e < 4; ++e) {
        const int row = m0 + acc_row<C>(i, e);
        if (row < a.M && col < a.L) O[(long long)row * a.L + col] = acc[i][j][e];
      }
    }
}

// Node sum fused into the last mode product: every block loops over all
// nodes b and keeps np <= PMAX running sums in registers.
template <class C, int PMAX>
__global__ __launch_bounds__(C::NT) void ttm_accum_kernel(TtmArgs a) {
  __shared__ double As[C::BM * C::LDK];
  __shared__ double Bs[C::BN * C::LDK];
  int m0, n0;
  tile_origin<C>(a.M, m0, n0);
  d4 y[PMAX][C::TM][C::TN];
#pragma unroll
  for (int q = 0; q < PMAX; ++q) zero_acc<C>(y[q]);
  for (int b = 0; b < a.nbatch; ++b) {
    d4 acc[C::TM][C::TN];
    zero_acc<C>(acc);
    tile_nt<C>(a.E + b * a.es, (const double*)a.X + b * a.xs, a.M, a.K, a.L, m0, n0, As, Bs, acc);
#pragma unroll
    for (int q = 0; q < PMAX; ++q) {
      if (q < a.np) {
        const double w = a.coef[q * a.ldcoef + b];
#pragma unroll
        for (int i = 0; i < C::TM; ++i)
#pragma unroll
          for (int j = 0; j < C::TN; ++j) y[q][i][j] += w * acc[i][j];
      }
    }
  }
#pragma unroll
  for (int q = 0; q < PMAX; ++q) {
    if (q < a.np) {
      double* Y = a.Y + q * a.ys;
#pragma unroll
      for (int i = 0; i < C::TM; ++i)
#pragma unroll
        for (int j = 0; j < C::TN; ++j) {
          const int col = n0 + acc_col<C>(j);
#pragma unroll
          for (int e = 0; e < 4; ++e) {
            const int row = m0 + acc_row<C>(i, e);
            if (row < a.M && col < a.L) Y[(long long)row * a.L + col] = y[q][i][j][e];
          }
        }
    }
  }
}

// Modified squaring fused into the last mode product (eq. squaring):
// batch b is order i = b+1, out = 2^{-i} (E y_i + sum_{j=1}^{i} y_j/(i-j)!).
template <class C>
__global__ __launch_bounds__(C::NT) void ttm_square_kernel(TtmArgs a) {
  __shared__ double As[C::BM * C::LDK];
  __shared__ double Bs[C::BN * C::LDK];
  int m0, n0;
  tile_origin<C>(a.M, m0, n0);
  const int b = blockIdx.y;
  d4 acc[C::TM][C::TN];
  zero_acc<C>(acc);
  tile_nt<C>(a.E + b * a.es, (const double*)a.X + b * a.xs, a.M, a.K, a.L, m0, n0, As, Bs, acc);
  const int order = b + 1;
  const double scale = ldexp(1.0, -order);
  double* O = (double*)a.O + b * a.os;
#pragma unroll
  for (int i = 0; i < C::TM; ++i)
#pragma unroll
    for (int j = 0; j < C::TN; ++j) {
      const int col = n0 + acc_col<C>(j);
#pragma unroll
      for (int e = 0; e < 4; ++e) {
        const int row = m0 + acc_row<C>(i, e);
        if (row < a.M && col < a.L) {
          const long long idx = (long long)row * a.L + col;
          double s = acc[i][j][e];
          double inv_fact = 1.0;  // 1/(i-j)! for j = i, i-1, ..., 1
          for (int jj = order; jj >= 1; --jj) {
            s += a.Yprev[(jj - 1) * a.yps + idx] * inv_fact;
            inv_fact /= (double)(order - jj + 1);
          }
          O[idx] = scale * s;
        }
      }
    }
}

// ---------------------------------------------------------------------------
// Small batched GEMM C = A B (n x n), one job per blockIdx.z.
// ---------------------------------------------------------------------------
template <class C>
__global__ __launch_bounds__(C::NT) void gemm_jobs_kernel(const GemmJob* __restrict__ jobs) {
  __shared__ double As[C::BM * C::LDK];
  __shared__ double Bs[C::BN * C::LDK];
  const GemmJob jb = jobs[blockIdx.z];
  const int m0 = blockIdx.x * C::BM, n0 = blockIdx.y * C::BN;
  if (m0 >= jb.n || n0 >= jb.n) return;  // uniform per block
  d4 acc[C::TM][C::TN];
  zero_acc<C>(acc);
  tile_nn<C>(jb.A, jb.B, jb.n, m0, n0, As, Bs, acc);
#pragma unroll
  for (int i = 0; i < C::TM; ++i)
#pragma unroll
    for (int j = 0; j < C::TN; ++j) {
      const int col = n0 + acc_col<C>(j);
#pragma unroll
      for (int e = 0; e < 4; ++e) {
        const int row = m0 + acc_row<C>(i, e);
        if (row < jb.n && col < jb.n) jb.C[(long long)row * jb.n + col] = acc[i][j][e];
      }
    }
}

__global__ void scale_jobs_kernel(const ScaleJob* __restrict__ jobs) {
  const ScaleJob jb = jobs[blockIdx.y];
  const long long nn = (long long)jb.n * jb.n;
  for (long long i = blockIdx.x * (long long)blockDim.x + threadIdx.x; i < nn; i += (long long)gridDim.x * blockDim.x)
    jb.dst[i] = jb.s * jb.src[i];
}

// dst[t] = I + sum_{k=1}^{K} c_t^k/k! Z^k by Horner's rule in c_t:
//   c (Z + c/2 (Z^2 + c/3 (Z^3 + ...))),
// with the K powers of one element held in registers for all targets.
__global__ __launch_bounds__(256) void taylor_jobs_kernel(const TaylorJob* __restrict__ jobs) {
  const TaylorJob& jb = jobs[blockIdx.y];
  const int n = jb.n, K = jb.K, nt = jb.nt;
  const long long nn = (long long)n * n;
  const double* __restrict__ Z = jb.Zpow;
  for (long long i = blockIdx.x * (long long)blockDim.x + threadIdx.x; i < nn; i += (long long)gridDim.x * blockDim.x) {
    double z[kMaxTaylorDegree];
#pragma unroll
    for (int k = 0; k < kMaxTaylorDegree; ++k) z[k] = (k < K) ? Z[k * nn + i] : 0.0;
    const double diag = (i / n == i % n) ? 1.0 : 0.0;
    for (int t = 0; t < nt; ++t) {
      const double c = jb.c[t];
      double s = 0.0;
#pragma unroll
      for (int k = kMaxTaylorDegree - 1; k >= 0; --k)
        if (k < K) s = z[k] + s * (c * (1.0 / (double)(k + 2)));
      jb.dst[t][i] = diag + c * s;
    }
  }
}

// ---------------------------------------------------------------------------
// Streaming helpers for the adaptive Clenshaw-Curtis path.
// ---------------------------------------------------------------------------
// partial[(blk * np + j) * 2 + 0] = max |y_j - yold_j|, [.. + 1] = max |y_j|
__global__ void absdiff_max_kernel(const double* __restrict__ y, const double* __restrict__ yold, int np,
                                   long long N, double* __restrict__ partial) {
  __shared__ double sd[256], sy[256];
  for (int j = 0; j < np; ++j) {
    double md = 0.0, my = 0.0;
    const double* yj = y + j * N;
    const double* oj = yold + j * N;
    for (long long i = blockIdx.x * (long long)blockDim.x + threadIdx.x; i < N; i += (long long)gridDim.x * blockDim.x) {
      const double v = yj[i];
      md = fmax(md, fabs(v - oj[i]));
      my = fmax(my, fabs(v));
    }
    sd[threadIdx.x] = md;
    sy[threadIdx.x] = my;
    __syncthreads();
    for (int s = blockDim.x / 2; s > 0; s >>= 1) {
      if ((int)threadIdx.x < s) {
        sd[threadIdx.x] = fmax(sd[threadIdx.x], sd[threadIdx.x + s]);
        sy[threadIdx.x] = fmax(sy[threadIdx.x], sy[threadIdx.x + s]);
      }
      __syncthreads();
    }
    if (threadIdx.x == 0) {
      partial[((long long)blockIdx.x * np + j) * 2 + 0] = sd[0];
      partial[((long long)blockIdx.x * np + j) * 2 + 1] = sy[0];
    }
    __syncthreads();
  }
}

// Y[j*N + i] = sum_b coef[j * ldcoef + b] * V_b[i], b running through the segments
__global__ void node_sum_kernel(NodeSegs segs, long long N, const double* __restrict__ coef, int ldcoef, int np,
                                double* __restrict__ Y) {
  for (long long i = blockIdx.x * (long long)blockDim.x + threadIdx.x; i < N; i += (long long)gridDim.x * blockDim.x) {
    double acc[PHIQ_MAX_P];
    for (int j = 0; j < np; ++j) acc[j] = 0.0;
    int b = 0;
    for (int sg = 0; sg < segs.nseg; ++sg) {
      const double* V = segs.V[sg];
      for (int c = 0; c < segs.count[sg]; ++c, ++b) {
        const double x = V[(long long)c * N + i];
        for (int j = 0; j < np; ++j) acc[j] += coef[j * ldcoef + b] * x;
      }
    }
    for (int j = 0; j < np; ++j) Y[j * N + i] = acc[j];
  }
}

// ---------------------------------------------------------------------------
// Launchers
// ---------------------------------------------------------------------------
namespace {
inline int cdiv(long long a, long long b) { return (int)((a + b - 1) / b); }
}  // namespace

int launch_gemm_jobs(const GemmJob* jobs, int njobs, int nmax, void* stream) {
  if (njobs <= 0) return hipSuccess;
  // few large-tile blocks would leave most CUs idle: use one-wave 32x32 tiles
  if ((long long)njobs * cdiv(nmax, 64) * cdiv(nmax, 64) < 512) {
    using C = Tile32;
    dim3 grid(cdiv(nmax, C::BM), cdiv(nmax, C::BN), njobs);
    hipLaunchKernelGGL(gemm_jobs_kernel<C>, grid, dim3(C::NT), 0, (hipStream_t)stream, jobs);
  } else {
    using C = Tile64;
    dim3 grid(cdiv(nmax, C::BM), cdiv(nmax, C::BN), njobs);
    hipLaunchKernelGGL(gemm_jobs_kernel<C>, grid, dim3(C::NT), 0, (hipStream_t)stream, jobs);
  }
  return hipGetLastError();
}

int launch_scale_jobs(const ScaleJob* jobs, int njobs, int nmax, void* stream) {
  if (njobs <= 0) return hipSuccess;
  dim3 grid(std::max(1, std::min(64, cdiv((long long)nmax * nmax, 256))), njobs);
  hipLaunchKernelGGL(scale_jobs_kernel, grid, dim3(256), 0, (hipStream_t)stream, jobs);
  return hipGetLastError();
}

int launch_taylor_jobs(const TaylorJob* jobs, int njobs, int nmax, void* stream) {
  if (njobs <= 0) return hipSuccess;
  dim3 grid(std::max(1, std::min(64, cdiv((long long)nmax * nmax, 256))), njobs);
  hipLaunchKernelGGL(taylor_jobs_kernel, grid, dim3(256), 0, (hipStream_t)stream, jobs);
  return hipGetLastError();
}

namespace {
template <class C>
dim3 ttm_grid(const TtmArgs& a, int nb) {
  return dim3((unsigned)cdiv(a.M, C::BM) * (unsigned)cdiv(a.L, C::BN), nb, 1);
}
}  // namespace

int launch_ttm_store(const TtmArgs& a, phiq_precision prec, void* stream) {
  if (prec != PHIQ_PREC_FP64) return launch_ttm_store_lowp(a, prec, stream);
  if (a.M > 64) {
    hipLaunchKernelGGL(ttm_store_kernel<Tile128>, ttm_grid<Tile128>(a, a.nbatch), dim3(Tile128::NT), 0,
                       (hipStream_t)stream, a);
  } else {
    hipLaunchKernelGGL(ttm_store_kernel<Tile64>, ttm_grid<Tile64>(a, a.nbatch), dim3(Tile64::NT), 0,
                       (hipStream_t)stream, a);
  }
  return hipGetLastError();
}

int launch_ttm_accum(const TtmArgs& a, phiq_precision prec, void* stream) {
  if (a.np > 4 || a.np < 1) return hipErrorInvalidValue;
  if (prec != PHIQ_PREC_FP64) return launch_ttm_accum_lowp(a, prec, stream);
  using C = Tile64;
  hipLaunchKernelGGL((ttm_accum_kernel<C, 4>), ttm_grid<C>(a, 1), dim3(C::NT), 0, (hipStream_t)stream, a);
  return hipGetLastError();
}

int launch_ttm_square(const TtmArgs& a, phiq_precision prec, void* stream) {
  if (prec != PHIQ_PREC_FP64) return launch_ttm_square_lowp(a, prec, stream);
  if (a.M > 64) {
    hipLaunchKernelGGL(ttm_square_kernel<Tile128>, ttm_grid<Tile128>(a, a.nbatch), dim3(Tile128::NT), 0,
                       (hipStream_t)stream, a);
  } else {
    hipLaunchKernelGGL(ttm_square_kernel<Tile64>, ttm_grid<Tile64>(a, a.nbatch), dim3(Tile64::NT), 0,
                       (hipStream_t)stream, a);
  }
  return hipGetLastError();
}

int launch_absdiff_max(const double* y, const double* yold, int np, long long N, double* partial, int nblocks,
                       void* stream) {
  hipLaunchKernelGGL(absdiff_max_kernel, dim3(nblocks), dim3(256), 0, (hipStream_t)stream, y, yold, np, N, partial);
  return hipGetLastError();
}

int launch_node_sum(const NodeSegs& segs, long long N, const double* coef, int ldcoef, int np, double* Y,
                    void* stream) {
  const int nb = std::max(1, std::min(4096, cdiv(N, 256)));
  hipLaunchKernelGGL(node_sum_kernel, dim3(nb), dim3(256), 0, (hipStream_t)stream, segs, N, coef, ldcoef, np, Y);
  return hipGetLastError();
}

}  // namespace phiq
