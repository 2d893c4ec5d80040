// FP64 MFMA tile building blocks shared by the mode-product kernels and the
// persistent batched kernel (gfx950, v_mfma_f64_16x16x4_f64).
//
//   A operand: lane l holds A[l % 16][l / 16]      (16 x 4)
//   B operand: lane l holds B[l / 16][l % 16]      (4 x 16)
//   D (4 doubles): lane l, element e holds D[l / 16 + 4 e][l % 16]
#pragma once

#include <hip/hip_runtime.h>

namespace phiq {

typedef double d4 __attribute__((ext_vector_type(4)));

// PAD: doubles of padding per LDS row (2 keeps rows 16-byte aligned for
// paired stores; 1 saves LDS so that one more block fits on a CU).
// MINW: waves per SIMD the kernels must allow (register budget), 1 = any.
template <int BM_, int BN_, int BK_, int WAVES_M_, int WAVES_N_, int PAD_ = 2, int MINW_ = 1>
struct Tile {
  static constexpr int BM = BM_, BN = BN_, BK = BK_;
  static constexpr int MINW = MINW_;
  static constexpr int WAVES_M = WAVES_M_, WAVES_N = WAVES_N_;
  static constexpr int NT = 64 * WAVES_M_ * WAVES_N_;
  static constexpr int WM = BM_ / WAVES_M_, WN = BN_ / WAVES_N_;
  static constexpr int TM = WM / 16, TN = WN / 16;
  static constexpr int LDK = BK_ + PAD_;  // padded row length in LDS (doubles)
  static constexpr int A_PER = BM_ * BK_ / NT;
  static constexpr int B_PER = BN_ * BK_ / NT;
  static_assert(A_PER * NT == BM_ * BK_ && B_PER * NT == BN_ * BK_, "tile not divisible");
  static_assert(TM * 16 == WM && TN * 16 == WN && BK_ % 4 == 0, "wave tile");
};

using Tile64 = Tile<64, 64, 16, 2, 2>;
using Tile128 = Tile<128, 64, 16, 2, 2>;
using Tile128x128 = Tile<128, 128, 16, 2, 2>;
using Tile256 = Tile<256, 64, 16, 4, 1>;
using Tile128k32 = Tile<128, 64, 32, 2, 2>;
using Tile64x128 = Tile<64, 128, 16, 2, 2>;
using Tile64k32 = Tile<64, 64, 32, 2, 2>;
using Tile128x128w8 = Tile<128, 128, 16, 4, 2>;  // 8 waves: fewer, larger blocks
using Tile32 = Tile<32, 32, 16, 1, 1>;
// one double of padding: 52 KB (64x128) / 35 KB (64x64) per block, so three
// (64x128, 128x64) or four (64x64) blocks fit in a CU's 160 KB of LDS
using Tile64x128p1 = Tile<64, 128, 16, 2, 2, 1, 3>;
using Tile128p1 = Tile<128, 64, 16, 2, 2, 1, 3>;
using Tile64p1 = Tile<64, 64, 16, 2, 2, 1>;
using Tile64x128p1r = Tile<64, 128, 16, 2, 2, 1>;  // the same without the register cap (fused epilogues)
// eight waves per block (32 x 32 or 32 x 16 per wave): fewer registers per
// wave, more waves per CU to hide latency
using Tile64x128p1w8 = Tile<64, 128, 16, 2, 4, 1>;
using Tile128p1w8 = Tile<128, 64, 16, 4, 2, 1>;
using Tile128x128p1 = Tile<128, 128, 16, 2, 2, 1, 2>;
using Tile64p1w8 = Tile<64, 64, 16, 2, 4, 1>;
using Tile64p1w8m2 = Tile<64, 64, 16, 2, 4, 1, 4>;  // the same within 128 registers: two blocks per CU

// ---------------------------------------------------------------------------
// Staging of rows [r0, r0+ROWS) x k-chunk [k0, k0+BK) of a row-major matrix
// with row length ld (k contiguous).
//
// Loads are branch-free and select nothing: lanes outside (rows_valid,
// k_valid) read a clamped in-range address, so a load's result is first
// needed when it is written to LDS one chunk later and the prefetch stays in
// flight during the MFMA work.  Rows past the end only feed outputs that are
// never stored; past the end of k the E operand is zeroed at the LDS store
// (ZK), which makes those products vanish whatever the X operand holds.
// With VEC (ld and k_valid even, 16-byte aligned base) lanes move pairs.
// ---------------------------------------------------------------------------
typedef double d2 __attribute__((ext_vector_type(2)));

template <int ROWS, int BK, int NT, int PER, bool VEC>
__device__ __forceinline__ void load_kmajor(const double* __restrict__ g, long long ld, int r0,
                                            int rows_valid, int k0, int k_valid, double (&reg)[PER]) {
  if constexpr (VEC) {
#pragma unroll
    for (int i = 0; i < PER / 2; ++i) {
      const int e = threadIdx.x + i * NT;
      const int row = r0 + e / (BK / 2), k = k0 + 2 * (e % (BK / 2));
      const int rc = row < rows_valid ? row : rows_valid - 1;
      const int kc = k < k_valid ? k : 0;
      const d2 v = *(const d2*)(g + (long long)rc * ld + kc);
      reg[2 * i] = v.x;
      reg[2 * i + 1] = v.y;
    }
  } else {
#pragma unroll
    for (int i = 0; i < PER; ++i) {
      const int e = threadIdx.x + i * NT;
      const int row = r0 + e / BK, k = k0 + e % BK;
      const int rc = row < rows_valid ? row : rows_valid - 1;
      const int kc = k < k_valid ? k : 0;
      reg[i] = g[(long long)rc * ld + kc];
    }
  }
}
template <int BK, int NT, int PER, int LDK, bool VEC, bool ZK>
__device__ __forceinline__ void store_kmajor(double* s, const double (&reg)[PER], int k0, int k_valid) {
  if constexpr (VEC) {
#pragma unroll
    for (int i = 0; i < PER / 2; ++i) {
      const int e = threadIdx.x + i * NT;
      const int r = e / (BK / 2), kk = 2 * (e % (BK / 2));
      const bool ok = !ZK || k0 + kk < k_valid;
      if constexpr (LDK % 2 == 0) {
        *(d2*)(s + r * LDK + kk) = ok ? (d2){reg[2 * i], reg[2 * i + 1]} : (d2){0.0, 0.0};
      } else {  // rows are only 8-byte aligned
        s[r * LDK + kk] = ok ? reg[2 * i] : 0.0;
        s[r * LDK + kk + 1] = ok ? reg[2 * i + 1] : 0.0;
      }
    }
  } else {
#pragma unroll
    for (int i = 0; i < PER; ++i) {
      const int e = threadIdx.x + i * NT;
      const bool ok = !ZK || k0 + e % BK < k_valid;
      s[(e / BK) * LDK + (e % BK)] = ok ? reg[i] : 0.0;
    }
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
    const bool ok = col < cols_valid && k < k_valid;
    const double v = g[(long long)(ok ? k : 0) * ld + (ok ? col : 0)];
    reg[i] = ok ? v : 0.0;
  }
}
// The same with pairs of columns per lane (ld and c0 even, 16-byte aligned
// base; cols_valid even, so a pair is valid or invalid as a whole).
template <int COLS, int BK, int NT, int PER>
__device__ __forceinline__ void load_nmajor_v(const double* __restrict__ g, long long ld, int c0, int cols_valid,
                                              int k0, int k_valid, double (&reg)[PER]) {
#pragma unroll
  for (int i = 0; i < PER / 2; ++i) {
    const int e = threadIdx.x + i * NT;
    const int kk = e / (COLS / 2), c = 2 * (e % (COLS / 2));
    const int k = k0 + kk, col = c0 + c;
    const bool ok = col < cols_valid && k < k_valid;
    const d2 v = *(const d2*)(g + (long long)(ok ? k : 0) * ld + (ok ? col : 0));
    reg[2 * i] = ok ? v.x : 0.0;
    reg[2 * i + 1] = ok ? v.y : 0.0;
  }
}
template <int COLS, int NT, int PER, int LDK>
__device__ __forceinline__ void store_nmajor_v(double* s, const double (&reg)[PER]) {
#pragma unroll
  for (int i = 0; i < PER / 2; ++i) {
    const int e = threadIdx.x + i * NT;
    const int kk = e / (COLS / 2), c = 2 * (e % (COLS / 2));
    s[c * LDK + kk] = reg[2 * i];
    s[(c + 1) * LDK + kk] = reg[2 * i + 1];
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

// acc += A[m0:m0+BM, :] * B[:, n0:n0+BN]  (A: n x n, B: n x n, row-major)
template <class C>
__device__ __forceinline__ void tile_nn(const double* __restrict__ A, const double* __restrict__ B, int n,
                                        int m0, int n0, double* As, double* Bs, d4 (&acc)[C::TM][C::TN]) {
  double ra[C::A_PER], rb[C::B_PER];
  load_kmajor<C::BM, C::BK, C::NT, C::A_PER, false>(A, n, m0, n, 0, n, ra);
  load_nmajor<C::BN, C::BK, C::NT, C::B_PER>(B, n, n0, n, 0, n, rb);
  for (int k0 = 0; k0 < n; k0 += C::BK) {
    __syncthreads();
    store_kmajor<C::BK, C::NT, C::A_PER, C::LDK, false, true>(As, ra, k0, n);
    store_nmajor<C::BN, C::NT, C::B_PER, C::LDK>(Bs, rb);
    __syncthreads();
    if (k0 + C::BK < n) {
      load_kmajor<C::BM, C::BK, C::NT, C::A_PER, false>(A, n, m0, n, k0 + C::BK, n, ra);
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

// acc += E[m0:m0+BM, :] X[n0:n0+BN, :]^T (E: M x K, X: L x K, row-major;
// with NN, X is K x L instead, element (j, k) at X[k * L + j]): register
// prefetch two chunks ahead and a double-buffered LDS tile, one barrier per
// K-chunk.  smem holds 2 (BM + BN) LDK doubles and is free when the call
// returns.

template <class C, bool VEC, bool NN = false>
__device__ __forceinline__ void tile_nt_db(const double* __restrict__ E, const double* __restrict__ X, int M, int K,
                                           int L, int m0, int n0, double* smem, d4 (&acc)[C::TM][C::TN]) {
  constexpr int STAGE = (C::BM + C::BN) * C::LDK;
  double ra[C::A_PER], rb[C::B_PER];
  const int nch = (K + C::BK - 1) / C::BK;
  auto load_b = [&](int k0) {
    if constexpr (NN && VEC)
      load_nmajor_v<C::BN, C::BK, C::NT, C::B_PER>(X, L, n0, L, k0, K, rb);
    else if constexpr (NN)
      load_nmajor<C::BN, C::BK, C::NT, C::B_PER>(X, L, n0, L, k0, K, rb);
    else
      load_kmajor<C::BN, C::BK, C::NT, C::B_PER, VEC>(X, K, n0, L, k0, K, rb);
  };
  auto store_b = [&](double* s, int k0) {
    if constexpr (NN && VEC)
      store_nmajor_v<C::BN, C::NT, C::B_PER, C::LDK>(s, rb);
    else if constexpr (NN)
      store_nmajor<C::BN, C::NT, C::B_PER, C::LDK>(s, rb);
    else
      store_kmajor<C::BK, C::NT, C::B_PER, C::LDK, VEC, false>(s, rb, k0, K);
  };
  load_kmajor<C::BM, C::BK, C::NT, C::A_PER, VEC>(E, K, m0, M, 0, K, ra);
  load_b(0);
  store_kmajor<C::BK, C::NT, C::A_PER, C::LDK, VEC, true>(smem, ra, 0, K);
  store_b(smem + C::BM * C::LDK, 0);
  if (nch > 1) {
    load_kmajor<C::BM, C::BK, C::NT, C::A_PER, VEC>(E, K, m0, M, C::BK, K, ra);
    load_b(C::BK);
  }
  __syncthreads();
  for (int c = 0; c < nch; ++c) {
    double* cur = smem + (c & 1) * STAGE;
    double* nxt = smem + ((c + 1) & 1) * STAGE;
    if (c + 1 < nch) {
      // readers of nxt (chunk c-1) passed the barrier at the end of c-1
      store_kmajor<C::BK, C::NT, C::A_PER, C::LDK, VEC, true>(nxt, ra, (c + 1) * C::BK, K);
      store_b(nxt + C::BM * C::LDK, (c + 1) * C::BK);
      if (c + 2 < nch) {
        load_kmajor<C::BM, C::BK, C::NT, C::A_PER, VEC>(E, K, m0, M, (c + 2) * C::BK, K, ra);
        load_b((c + 2) * C::BK);
      }
    }
    mma_chunk<C>(cur, cur + C::BM * C::LDK, acc);
    __syncthreads();
  }
}

template <class C>
__host__ __device__ inline long long ttm_tiles(int M, int L, int nb) {
  return (long long)((M + C::BM - 1) / C::BM) * ((L + C::BN - 1) / C::BN) * nb;
}

}  // namespace phiq
