// Batched phi-actions: one launch per dependency level, each over every
// problem of the batch (gfx950).
//
// The host splits every problem into stages (1D exponentials: powers, Taylor
// sums, squarings; per vector: node chains with the node sum, modified
// squaring steps, phi_0), gives each stage its depth in the dependency
// graph and stores the stages by depth.  One launch covers all tiles of one
// depth, across all problems, so small and large problems fill the GPU
// together and the kernel boundary orders the depths.  Workgroups never
// wait on each other: each takes tiles with a grid-stride loop and exits.
#include <hip/hip_runtime.h>

#include "phiq_internal.h"
#include "tile_fp64.h"

namespace phiq {

using BT = Tile<kBatchTile, kBatchTile, 16, 2, 2>;  // 256 threads, 64 x 64 output tiles
static_assert(BT::NT == 256, "batch worker size");

namespace {

template <class C>
__device__ __forceinline__ void store_tile(double* O, int M, int L, int m0, int n0, const d4 (&acc)[C::TM][C::TN]) {
#pragma unroll
  for (int i = 0; i < C::TM; ++i)
#pragma unroll
    for (int j = 0; j < C::TN; ++j) {
      const int col = n0 + acc_col<C>(j);
#pragma unroll
      for (int e = 0; e < 4; ++e) {
        const int row = m0 + acc_row<C>(i, e);
        if (row < M && col < L) O[(long long)row * L + col] = acc[i][j][e];
      }
    }
}

__device__ void run_gemm(const BatchStage& S, int tile, double* smem) {
  const int n = S.M;
  const int mt = (n + BT::BM - 1) / BT::BM;
  const int m0 = (tile % mt) * BT::BM, n0 = (tile / mt) * BT::BN;
  d4 acc[BT::TM][BT::TN];
  zero_acc<BT>(acc);
  tile_nn<BT>(S.E, S.X, n, m0, n0, smem, smem + BT::BM * BT::LDK, acc);
  store_tile<BT>(S.O, n, n, m0, n0, acc);
}

// Same Horner form as the single-problem Taylor kernel, one element at a time.
__device__ void run_taylor(const BatchTaylor& jb, int tile) {
  const int n = jb.n, K = jb.K, nt = jb.nt;
  const long long nn = (long long)n * n;
  for (int r = 0; r < kBatchTaylorChunk / 256; ++r) {
    const long long i = (long long)tile * kBatchTaylorChunk + r * 256 + threadIdx.x;
    if (i >= nn) break;
    double z[kMaxTaylorDegree];
#pragma unroll
    for (int k = 0; k < kMaxTaylorDegree; ++k)
      z[k] = (k < K) ? (k == 0 ? jb.Z1[i] : jb.Zp[(k - 1) * nn + i]) : 0.0;
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

template <bool VEC>
__device__ void run_store(const BatchStage& S, int tile, double* smem) {
  const int mt = (S.M + BT::BM - 1) / BT::BM;
  const int m0 = (tile % mt) * BT::BM;
  const int r = tile / mt;
  const int b = r % S.nb;
  const int n0 = (r / S.nb) * BT::BN;
  d4 acc[BT::TM][BT::TN];
  zero_acc<BT>(acc);
  tile_nt_db<BT, VEC>(S.E + b * S.es, S.X + b * S.xs, S.M, S.K, S.L, m0, n0, smem, acc);
  store_tile<BT>(S.O + b * S.os, S.M, S.L, m0, n0, acc);
}

template <bool VEC>
__device__ void run_accum(const BatchStage& S, int tile, double* smem) {
  const int mt = (S.M + BT::BM - 1) / BT::BM;
  const int m0 = (tile % mt) * BT::BM, n0 = (tile / mt) * BT::BN;
  d4 y[4][BT::TM][BT::TN];
#pragma unroll
  for (int q = 0; q < 4; ++q) zero_acc<BT>(y[q]);
  for (int b = 0; b < S.nb; ++b) {
    d4 acc[BT::TM][BT::TN];
    zero_acc<BT>(acc);
    tile_nt_db<BT, VEC>(S.E + b * S.es, S.X + b * S.xs, S.M, S.K, S.L, m0, n0, smem, acc);
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      const double w = q < S.np ? S.coef[q * S.ldcoef + b] : 0.0;
#pragma unroll
      for (int i = 0; i < BT::TM; ++i)
#pragma unroll
        for (int j = 0; j < BT::TN; ++j) y[q][i][j] += w * acc[i][j];
    }
  }
#pragma unroll
  for (int q = 0; q < 4; ++q) {
    if (q >= S.np) break;
    double* Y = S.Y + q * S.ys;
#pragma unroll
    for (int i = 0; i < BT::TM; ++i)
#pragma unroll
      for (int j = 0; j < BT::TN; ++j) {
        const int col = n0 + acc_col<BT>(j);
#pragma unroll
        for (int e = 0; e < 4; ++e) {
          const int row = m0 + acc_row<BT>(i, e);
          if (row < S.M && col < S.L) {
            const long long idx = (long long)row * S.L + col;
            Y[idx] = S.accumulate ? Y[idx] + y[q][i][j][e] : y[q][i][j][e];
          }
        }
      }
  }
}

// All orders of one modified-squaring step (eq. squaring), np <= 4.  The
// y_j tiles are re-read for each order (they stay in L2) rather than held in
// registers, which keeps the worker within two waves per SIMD.
__constant__ double kInvFact[4] = {1.0, 1.0, 0.5, 1.0 / 6.0};

template <bool VEC>
__device__ void run_square(const BatchStage& S, int tile, double* smem) {
  const int mt = (S.M + BT::BM - 1) / BT::BM;
  const int m0 = (tile % mt) * BT::BM, n0 = (tile / mt) * BT::BN;
  for (int i = 0; i < S.np; ++i) {
    d4 acc[BT::TM][BT::TN];
    zero_acc<BT>(acc);
    tile_nt_db<BT, VEC>(S.E, S.X + i * S.xs, S.M, S.K, S.L, m0, n0, smem, acc);
    const double scale = ldexp(1.0, -(i + 1));
    double* O = S.O + i * S.os;
#pragma unroll
    for (int ti = 0; ti < BT::TM; ++ti)
#pragma unroll
      for (int tj = 0; tj < BT::TN; ++tj) {
        const int col = n0 + acc_col<BT>(tj);
#pragma unroll
        for (int e = 0; e < 4; ++e) {
          const int row = m0 + acc_row<BT>(ti, e);
          if (row < S.M && col < S.L) {
            const long long idx = (long long)row * S.L + col;
            double s = acc[ti][tj][e];
            for (int j = 0; j <= i; ++j) s += S.Y[j * S.ys + idx] * kInvFact[i - j];
            O[idx] = scale * s;
          }
        }
      }
  }
}

__global__ __launch_bounds__(256, 2) void batch_level_kernel(BatchArgs a) {
  __shared__ double smem[2 * (BT::BM + BT::BN) * BT::LDK];
  for (long long g = a.tile_begin + blockIdx.x; g < a.tile_end; g += gridDim.x) {
    int lo = 0, hi = a.nstages - 1;  // last stage with tile0 <= g (block-uniform)
    while (lo < hi) {
      const int mid = (lo + hi + 1) >> 1;
      if (a.st[mid].tile0 <= g) lo = mid; else hi = mid - 1;
    }
    const BatchStage& S = a.st[lo];
    const int tile = (int)(g - S.tile0);
    switch (S.type) {
      case kStageGemm: run_gemm(S, tile, smem); break;
      case kStageTaylor: run_taylor(a.tj[S.aux], tile); break;
      case kStageStore:
        if (S.vec) run_store<true>(S, tile, smem); else run_store<false>(S, tile, smem);
        break;
      case kStageAccum:
        if (S.vec) run_accum<true>(S, tile, smem); else run_accum<false>(S, tile, smem);
        break;
      default:
        if (S.vec) run_square<true>(S, tile, smem); else run_square<false>(S, tile, smem);
        break;
    }
    __syncthreads();  // smem is reused by the next tile
  }
}

}  // namespace

int batch_workers(int* blocks) {
  int dev = 0, cus = 0, per = 0;
  hipError_t e = hipGetDevice(&dev);
  if (e == hipSuccess) e = hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev);
  if (e == hipSuccess) e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&per, batch_level_kernel, 256, 0);
  if (e != hipSuccess) return e;
  *blocks = cus * (per > 0 ? per : 1);
  return hipSuccess;
}

int launch_batch_level(const BatchArgs& a, int blocks, void* stream) {
  hipLaunchKernelGGL(batch_level_kernel, dim3(blocks), dim3(256), 0, (hipStream_t)stream, a);
  return hipGetLastError();
}

}  // namespace phiq
