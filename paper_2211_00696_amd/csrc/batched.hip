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

#include <algorithm>

#include "phiq_internal.h"
#include "tile_fp64.h"

namespace phiq {

using BT = Tile<kBatchTile, kBatchTile, 16, 2, 2>;  // 256 threads, 64 x 64 output tiles
using BW = Tile<kBatchTile, kBatchWideN, 16, 2, 4, 1>;  // wide stores: 512 threads, 64 x 128 tiles
using B8 = Tile<kBatchTile, kBatchTile, 16, 2, 4, 1>;   // wide node sums / squaring: 512 threads, 64 x 64
constexpr int kXcdCount = 8;
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

__device__ __forceinline__ void run_gemm(const BatchStage& S, int tile, double* smem) {
  const int n = S.M;
  const int mt = (n + BT::BM - 1) / BT::BM;
  const int m0 = (tile % mt) * BT::BM, n0 = (tile / mt) * BT::BN;
  d4 acc[BT::TM][BT::TN];
  zero_acc<BT>(acc);
  tile_nn<BT>(S.E, S.X, n, m0, n0, smem, smem + BT::BM * BT::LDK, acc);
  store_tile<BT>(S.O, n, n, m0, n0, acc);
}

// Same Horner form as the single-problem Taylor kernel, one element at a time.
__device__ __forceinline__ void run_taylor(const BatchTaylor& jb, int tile) {
  const int n = jb.n, K = jb.K, nt = jb.nt;
  const long long nn = (long long)n * n;
  for (int r = 0; r < kBatchTaylorChunk / (int)blockDim.x; ++r) {  // 256 or 512 threads
    const long long i = (long long)tile * kBatchTaylorChunk + r * (int)blockDim.x + threadIdx.x;
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
__device__ __forceinline__ void run_store(const BatchStage& S, int tile, double* smem) {
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
__device__ __forceinline__ void run_store_wide(const BatchStage& S, int tile, double* smem) {
  const int mt = (S.M + BW::BM - 1) / BW::BM;
  const int m0 = (tile % mt) * BW::BM;
  const int r = tile / mt;
  const int b = r % S.nb;
  const int n0 = (r / S.nb) * BW::BN;
  d4 acc[BW::TM][BW::TN];
  zero_acc<BW>(acc);
  tile_nt_db<BW, VEC>(S.E + b * S.es, S.X + b * S.xs, S.M, S.K, S.L, m0, n0, smem, acc);
  store_tile<BW>(S.O + b * S.os, S.M, S.L, m0, n0, acc);
}

template <class C, int NP, bool VEC>
__device__ __forceinline__ void run_accum(const BatchStage& S, int tile, double* smem) {
  const int mt = (S.M + C::BM - 1) / C::BM;
  const int m0 = (tile % mt) * C::BM, n0 = (tile / mt) * C::BN;
  d4 y[NP][C::TM][C::TN];
#pragma unroll
  for (int q = 0; q < NP; ++q) zero_acc<C>(y[q]);
  for (int b = 0; b < S.nb; ++b) {
    d4 acc[C::TM][C::TN];
    zero_acc<C>(acc);
    tile_nt_db<C, VEC>(S.E + b * S.es, S.X + b * S.xs, S.M, S.K, S.L, m0, n0, smem, acc);
#pragma unroll
    for (int q = 0; q < NP; ++q) {
      const double w = S.coef[q * S.ldcoef + b];
#pragma unroll
      for (int i = 0; i < C::TM; ++i)
#pragma unroll
        for (int j = 0; j < C::TN; ++j) y[q][i][j] += w * acc[i][j];
    }
  }
#pragma unroll
  for (int q = 0; q < NP; ++q) {
    double* Y = S.Y + q * S.ys;
#pragma unroll
    for (int i = 0; i < C::TM; ++i)
#pragma unroll
      for (int j = 0; j < C::TN; ++j) {
        const int col = n0 + acc_col<C>(j);
#pragma unroll
        for (int e = 0; e < 4; ++e) {
          const int row = m0 + acc_row<C>(i, e);
          if (row < S.M && col < S.L) {
            const long long idx = (long long)row * S.L + col;
            Y[idx] = S.accumulate ? Y[idx] + y[q][i][j][e] : y[q][i][j][e];
          }
        }
      }
  }
}

// All NP orders of one modified-squaring step (eq. squaring), NP <= 4: the
// block computes E y_i for i = 1..NP in turn; each y_i tile is loaded (into
// registers, before its product's K loop so that the load overlaps it) once
// and kept for the later orders.
template <class C, int NP, bool VEC>
__device__ __forceinline__ void run_square(const BatchStage& S, int tile, double* smem) {
  const int mt = (S.M + C::BM - 1) / C::BM;
  const int m0 = (tile % mt) * C::BM, n0 = (tile / mt) * C::BN;
  const double ifact[4] = {1.0, 1.0, 0.5, 1.0 / 6.0};
  d4 ys[NP][C::TM][C::TN];
#pragma unroll
  for (int i = 0; i < NP; ++i) {
#pragma unroll
    for (int ti = 0; ti < C::TM; ++ti)
#pragma unroll
      for (int tj = 0; tj < C::TN; ++tj) {
        const int col = n0 + acc_col<C>(tj);
#pragma unroll
        for (int e = 0; e < 4; ++e) {
          const int row = m0 + acc_row<C>(ti, e);
          const int rc = row < S.M ? row : S.M - 1, cc = col < S.L ? col : S.L - 1;
          ys[i][ti][tj][e] = S.Y[i * S.ys + (long long)rc * S.L + cc];
        }
      }
    d4 acc[C::TM][C::TN];
    zero_acc<C>(acc);
    tile_nt_db<C, VEC>(S.E, S.X + i * S.xs, S.M, S.K, S.L, m0, n0, smem, acc);
    const double scale = ldexp(1.0, -(i + 1));
    double* O = S.O + i * S.os;
#pragma unroll
    for (int ti = 0; ti < C::TM; ++ti)
#pragma unroll
      for (int tj = 0; tj < C::TN; ++tj) {
        const int col = n0 + acc_col<C>(tj);
#pragma unroll
        for (int e = 0; e < 4; ++e) {
          const int row = m0 + acc_row<C>(ti, e);
          double s = acc[ti][tj][e];
#pragma unroll
          for (int j = 0; j <= i; ++j) s += ys[j][ti][tj][e] * ifact[i - j];
          if (row < S.M && col < S.L) O[(long long)row * S.L + col] = scale * s;
        }
      }
  }
}

// One launch: the tiles [tile_begin, tile_end) of stages [stage_begin,
// stage_end), all of type TYPE.  The launch's tiles are dealt XCD-aware: the
// hardware gives consecutive workgroups to the 8 XCDs in turn, so the
// workgroups of one XCD take one contiguous eighth of the tiles (the tiles
// of one stage that read the same operand rows are adjacent) and share its
// L2.  Each workgroup walks its tiles with a stride of the grid size.
template <int TYPE, int NP, bool VEC>
__global__ __launch_bounds__(256) void batch_kernel(BatchArgs a) {
  __shared__ double smem[(TYPE == kStageTaylor) ? 1 : 2 * (BT::BM + BT::BN) * BT::LDK];
  const long long T = a.tile_end - a.tile_begin;
  const long long per = (T + kXcdCount - 1) / kXcdCount;
  const int xcd = blockIdx.x % kXcdCount;
  const long long G = gridDim.x / kXcdCount;  // workgroups per XCD (grid is a multiple of 8)
  int lo = a.stage_begin;
  for (long long v = blockIdx.x / kXcdCount; v < per; v += G) {
    const long long t = (long long)xcd * per + v;
    if (t >= T) break;
    const long long g = a.tile_begin + t;
    int hi = a.stage_end - 1;  // last stage with tile0 <= g; g only grows, so lo only grows
    while (lo < hi) {
      const int mid = (lo + hi + 1) >> 1;
      if (a.st[mid].tile0 <= g) lo = mid; else hi = mid - 1;
    }
    const BatchStage& S = a.st[lo];
    const int tile = (int)(g - S.tile0);
    if constexpr (TYPE == kStageGemm) {
      run_gemm(S, tile, smem);
    } else if constexpr (TYPE == kStageTaylor) {
      run_taylor(a.tj[S.aux], tile);
    } else if constexpr (TYPE == kStageStore) {
      run_store<VEC>(S, tile, smem);
    } else if constexpr (TYPE == kStageAccum) {
      run_accum<BT, NP, VEC>(S, tile, smem);
    } else {
      run_square<BT, NP, VEC>(S, tile, smem);
    }
    __syncthreads();  // smem is reused by the next tile
  }
}

// The wide stage types: the same tile walk with 512-thread workgroups.
template <int TYPE, int NP, bool VEC>
__global__ __launch_bounds__(512) void batch_wide_kernel(BatchArgs a) {
  __shared__ double smem[TYPE == kStageStoreWide ? 2 * (BW::BM + BW::BN) * BW::LDK : 2 * (B8::BM + B8::BN) * B8::LDK];
  const long long T = a.tile_end - a.tile_begin;
  const long long per = (T + kXcdCount - 1) / kXcdCount;
  const int xcd = blockIdx.x % kXcdCount;
  const long long G = gridDim.x / kXcdCount;
  int lo = a.stage_begin;
  for (long long v = blockIdx.x / kXcdCount; v < per; v += G) {
    const long long t = (long long)xcd * per + v;
    if (t >= T) break;
    const long long g = a.tile_begin + t;
    int hi = a.stage_end - 1;
    while (lo < hi) {
      const int mid = (lo + hi + 1) >> 1;
      if (a.st[mid].tile0 <= g) lo = mid; else hi = mid - 1;
    }
    const BatchStage& S = a.st[lo];
    const int tile = (int)(g - S.tile0);
    if constexpr (TYPE == kStageStoreWide) {
      run_store_wide<VEC>(S, tile, smem);
    } else if constexpr (TYPE == kStageAccumWide) {
      run_accum<B8, NP, VEC>(S, tile, smem);
    } else {
      run_square<B8, NP, VEC>(S, tile, smem);
    }
    __syncthreads();  // smem is reused by the next tile
  }
}

// ---------------------------------------------------------------------------
// One persistent launch for the whole batch.  Workgroups of 512 threads take
// tiles one at a time from a global counter, in the global order of the
// schedule (depth by depth), so every tile a tile depends on has a smaller
// number and was taken earlier by a workgroup that is running; the workgroup
// holding the smallest unfinished tile always has its inputs complete, so
// the batch finishes whatever number of workgroups is resident (no
// co-residency is assumed).  A tile first waits until every group it reads
// is complete (per-group completion counters, loaded with acquire semantics
// at device scope so the producers' results are visible across XCDs), runs
// with the eight-wave tiles (64 x 64 outputs like the four-wave ones, so the
// schedule's tile counts hold; wide stores keep their 64 x 128 tiles), and
// counts itself done with a release at device scope.  Every wait is bounded:
// after spin_limit polls it sets ctl->err and the workgroup stops, and the
// others stop at their next poll, so the kernel always ends.
// ---------------------------------------------------------------------------
// returns false when the wait gave up or another one did
__device__ bool wait_group(const BatchPersistArgs& p, int w, int need) {
  if (w < 0) return true;
  for (long long it = 0;; ++it) {
    const unsigned c = __hip_atomic_load(p.done + w, __ATOMIC_ACQUIRE, __HIP_MEMORY_SCOPE_AGENT);
    if (c >= (unsigned)need) return true;
    if (__hip_atomic_load(&p.ctl->err, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT)) return false;
    if (it >= p.spin_limit) {
      __hip_atomic_store(&p.ctl->err, 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
      return false;
    }
    __builtin_amdgcn_s_sleep(4);
  }
}

template <class C, int NP>
__device__ __forceinline__ void accum_vec(const BatchStage& S, int tile, double* smem) {
  if (S.vec)
    run_accum<C, NP, true>(S, tile, smem);
  else
    run_accum<C, NP, false>(S, tile, smem);
}
template <class C, int NP>
__device__ __forceinline__ void square_vec(const BatchStage& S, int tile, double* smem) {
  if (S.vec)
    run_square<C, NP, true>(S, tile, smem);
  else
    run_square<C, NP, false>(S, tile, smem);
}

__device__ __forceinline__ void run_gemm8(const BatchStage& S, int tile, double* smem) {
  const int n = S.M;
  const int mt = (n + B8::BM - 1) / B8::BM;
  const int m0 = (tile % mt) * B8::BM, n0 = (tile / mt) * B8::BN;
  d4 acc[B8::TM][B8::TN];
  zero_acc<B8>(acc);
  tile_nn<B8>(S.E, S.X, n, m0, n0, smem, smem + B8::BM * B8::LDK, acc);
  store_tile<B8>(S.O, n, n, m0, n0, acc);
}

template <bool VEC>
__device__ __forceinline__ void run_store8(const BatchStage& S, int tile, double* smem) {
  const int mt = (S.M + B8::BM - 1) / B8::BM;
  const int m0 = (tile % mt) * B8::BM;
  const int r = tile / mt;
  const int b = r % S.nb;
  const int n0 = (r / S.nb) * B8::BN;
  d4 acc[B8::TM][B8::TN];
  zero_acc<B8>(acc);
  tile_nt_db<B8, VEC>(S.E + b * S.es, S.X + b * S.xs, S.M, S.K, S.L, m0, n0, smem, acc);
  store_tile<B8>(S.O + b * S.os, S.M, S.L, m0, n0, acc);
}

__device__ __forceinline__ void run_any(const BatchArgs& a, const BatchStage& S, int tile, double* smem) {
  switch (S.type) {
    case kStageGemm: run_gemm8(S, tile, smem); break;
    case kStageTaylor: run_taylor(a.tj[S.aux], tile); break;
    case kStageStore:
      if (S.vec) run_store8<true>(S, tile, smem); else run_store8<false>(S, tile, smem);
      break;
    case kStageStoreWide:
      if (S.vec) run_store_wide<true>(S, tile, smem); else run_store_wide<false>(S, tile, smem);
      break;
    case kStageAccum:
    case kStageAccumWide:
      switch (S.np) {
        case 1: accum_vec<B8, 1>(S, tile, smem); break;
        case 2: accum_vec<B8, 2>(S, tile, smem); break;
        case 3: accum_vec<B8, 3>(S, tile, smem); break;
        default: accum_vec<B8, 4>(S, tile, smem); break;
      }
      break;
    default:
      switch (S.np) {
        case 1: square_vec<B8, 1>(S, tile, smem); break;
        case 2: square_vec<B8, 2>(S, tile, smem); break;
        case 3: square_vec<B8, 3>(S, tile, smem); break;
        default: square_vec<B8, 4>(S, tile, smem); break;
      }
  }
}

// Tiles are taken kPersistChunk at a time (one atomic on the shared counter
// per chunk instead of per tile: that counter and the completion counters
// are the kernel's only contended addresses), and a chunk's tiles run in
// order.  A workgroup waits only when the stage changes (tiles of one stage
// do not read each other), and publishes the completions it holds for a
// group when the group changes, before any wait and at the end of its chunk,
// so it never waits while holding completions that another workgroup may
// need: the workgroup with the smallest unfinished tile still finds its
// inputs published or about to be.
constexpr int kPersistChunk = 32;

__global__ __launch_bounds__(512) void batch_persistent_kernel(BatchArgs a, BatchPersistArgs p) {
  __shared__ double smem[2 * (BW::BM + BW::BN) * BW::LDK];
  __shared__ long long sh_base;
  __shared__ int sh_ok;
  int lo = 0;
  int ready = -1;      // stage whose inputs were found complete
  int pend_sig = -1;   // thread 0: group of the completions not yet published
  unsigned pend = 0;   // thread 0: their number
  auto publish = [&]() {
    if (threadIdx.x == 0 && pend) {
      __hip_atomic_fetch_add(p.done + pend_sig, pend, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_AGENT);
      pend = 0;
    }
  };
  for (;;) {
    if (threadIdx.x == 0)
      sh_base = (long long)__hip_atomic_fetch_add(&p.ctl->next, (unsigned long long)kPersistChunk, __ATOMIC_RELAXED,
                                                  __HIP_MEMORY_SCOPE_AGENT);
    __syncthreads();
    const long long base = sh_base;  // thread 0 rewrites it only after the barrier that ends a tile
    if (base >= p.total) break;
    const long long end = std::min(base + (long long)kPersistChunk, p.total);
    bool ok = true;
    for (long long g = base; g < end; ++g) {
      int hi = p.nstages - 1;  // last stage with tile0 <= g; g only grows, so lo only grows
      while (lo < hi) {
        const int mid = (lo + hi + 1) >> 1;
        if (a.st[mid].tile0 <= g) lo = mid; else hi = mid - 1;
      }
      const BatchStage& S = a.st[lo];
      if (lo != ready) {
        publish();
        if (threadIdx.x == 0) sh_ok = wait_group(p, S.wait0, S.need0) && wait_group(p, S.wait1, S.need1);
        __syncthreads();
        if (!sh_ok) {
          ok = false;
          break;
        }
        ready = lo;
      }
      run_any(a, S, (int)(g - S.tile0), smem);
      __syncthreads();  // every thread's results are written (and smem is free)
      if (threadIdx.x == 0) {
        if (pend_sig != S.signal) publish();
        pend_sig = S.signal;
        ++pend;
      }
    }
    publish();
    if (!ok) break;
  }
}

template <int TYPE, int NP>
hipError_t launch_wide(const BatchArgs& a, bool vec, dim3 grid, hipStream_t st) {
  if (vec)
    hipLaunchKernelGGL((batch_wide_kernel<TYPE, NP, true>), grid, dim3(512), 0, st, a);
  else
    hipLaunchKernelGGL((batch_wide_kernel<TYPE, NP, false>), grid, dim3(512), 0, st, a);
  return hipGetLastError();
}

template <int TYPE>
hipError_t launch_wide_type(const BatchArgs& a, int np, bool vec, dim3 grid, hipStream_t st) {
  switch (np) {
    case 1: return launch_wide<TYPE, 1>(a, vec, grid, st);
    case 2: return launch_wide<TYPE, 2>(a, vec, grid, st);
    case 3: return launch_wide<TYPE, 3>(a, vec, grid, st);
    case 4: return launch_wide<TYPE, 4>(a, vec, grid, st);
    default: return hipErrorInvalidValue;
  }
}

template <int TYPE, int NP>
hipError_t launch_np(const BatchArgs& a, bool vec, dim3 grid, hipStream_t st) {
  if (vec)
    hipLaunchKernelGGL((batch_kernel<TYPE, NP, true>), grid, dim3(256), 0, st, a);
  else
    hipLaunchKernelGGL((batch_kernel<TYPE, NP, false>), grid, dim3(256), 0, st, a);
  return hipGetLastError();
}

template <int TYPE>
hipError_t launch_type(const BatchArgs& a, int np, bool vec, dim3 grid, hipStream_t st) {
  switch (np) {
    case 1: return launch_np<TYPE, 1>(a, vec, grid, st);
    case 2: return launch_np<TYPE, 2>(a, vec, grid, st);
    case 3: return launch_np<TYPE, 3>(a, vec, grid, st);
    case 4: return launch_np<TYPE, 4>(a, vec, grid, st);
    default: return hipErrorInvalidValue;
  }
}

}  // namespace

int launch_batch_persistent(const BatchArgs& a, const BatchPersistArgs& p, void* stream) {
  hipStream_t st = (hipStream_t)stream;
  static int per_cu = 0;
  if (!per_cu) {
    int b = 0;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&b, batch_persistent_kernel, 512, 0) != hipSuccess || b < 1)
      b = 1;
    per_cu = b;
  }
  int dev = 0, cus = 256;
  if (hipGetDevice(&dev) != hipSuccess || hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess)
    cus = 256;
  // co-resident workgroups (not needed for progress: tiles are handed out in
  // dependency order), at most one per tile
  const long long g = std::min<long long>((long long)cus * per_cu, std::max<long long>(1, p.total));
  hipLaunchKernelGGL(batch_persistent_kernel, dim3((unsigned)g), dim3(512), 0, st, a, p);
  return hipGetLastError();
}

int launch_batch(const BatchArgs& a, int type, int np, int vec, int blocks, void* stream) {
  const dim3 grid(blocks);
  hipStream_t st = (hipStream_t)stream;
  switch (type) {
    case kStageGemm:
      hipLaunchKernelGGL((batch_kernel<kStageGemm, 0, false>), grid, dim3(256), 0, st, a);
      return hipGetLastError();
    case kStageTaylor:
      hipLaunchKernelGGL((batch_kernel<kStageTaylor, 0, false>), grid, dim3(256), 0, st, a);
      return hipGetLastError();
    case kStageStore: return launch_np<kStageStore, 0>(a, vec != 0, grid, st);
    case kStageStoreWide: return launch_wide<kStageStoreWide, 0>(a, vec != 0, grid, st);
    case kStageAccumWide: return launch_wide_type<kStageAccumWide>(a, np, vec != 0, grid, st);
    case kStageSquareWide: return launch_wide_type<kStageSquareWide>(a, np, vec != 0, grid, st);
    case kStageAccum: return launch_type<kStageAccum>(a, np, vec != 0, grid, st);
    case kStageSquare: return launch_type<kStageSquare>(a, np, vec != 0, grid, st);
    default: return hipErrorInvalidValue;
  }
}

}  // namespace phiq
