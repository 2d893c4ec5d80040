// Split-bf16 mode products with the 1D factor resident in LDS (gfx950).
//
//   out[i][j] = sum_k E[i][k] X[j][k],  i < M = K = n,  j < L,
//
// formed as hi_E hi_X + hi_E lo_X + lo_E hi_X on v_mfma_f32_16x16x32_bf16
// with FP32 accumulation (x = hi + lo, hi = bf16(x), lo = bf16(x - hi)).
//
// Why a second kernel: the general tile kernel (kernels_lowp.hip) stages a
// 128 x 32 panel of E and a 64 x 32 panel of X through LDS per 32-deep
// chunk with a barrier each time, so every tile re-reads E from L2 and only
// two chunks of loads are in flight; at n = 256 it moves 2 TB/s.  Here:
//   * A block keeps BM rows of E (bf16 hi and lo, BM x K x 4 bytes: 128 KB
//     at n = 256) in LDS for as long as it works with that factor, in MFMA
//     fragment order (each lane's 16-byte operand is contiguous, so the
//     reads are free of bank conflicts).
//   * Waves stream X from global memory straight into registers: a wave
//     owns 16 TN columns of the output (rows of X) and walks K in 64-deep
//     steps; each lane loads 16 consecutive k of one column (64 bytes FP32,
//     128 bytes FP64) and splits them into hi/lo itself.  PF steps of loads
//     are in flight, and the ring runs on across tile boundaries, so a
//     wave's memory pipeline never drains between tiles.  No barrier in the
//     steady state.
//   * Inside a 64-deep step the k order is permuted in both operands alike:
//     lane group g (= lane / 16) of MFMA step s covers k = 16 g + 8 s + 0..7.
//     The sum over k is unchanged.
//   * Persistent blocks take contiguous ranges of work units (factor b, row
//     half h, column tile), factor-major, so a block reloads E rarely.  With
//     two row halves (n = 256) the two blocks of a pair run on one XCD
//     (ids k and k + 8) and take the same column tiles, so the second read
//     of an X tile comes from that XCD's L2.
// Used for n in {64, 128, 256} (K a multiple of 64, M = K); other shapes
// take the general kernel.
#include <hip/hip_ext.h>
#include <hip/hip_runtime.h>

#include "phiq_internal.h"

namespace phiq {

#define PHIQ_LAUNCH_R(K, G, B, SH, ST, ...)                                                               \
  do {                                                                                                    \
    if (g_launch_events[0])                                                                               \
      hipExtLaunchKernelGGL(K, G, B, SH, ST, (hipEvent_t)g_launch_events[0], (hipEvent_t)g_launch_events[1], \
                            0, __VA_ARGS__);                                                              \
    else                                                                                                  \
      hipLaunchKernelGGL(K, G, B, SH, ST, __VA_ARGS__);                                                   \
  } while (0)

namespace {

typedef float f4 __attribute__((ext_vector_type(4)));
typedef __bf16 bf8 __attribute__((ext_vector_type(8)));
typedef double dv2 __attribute__((ext_vector_type(2)));

constexpr int kXcd = 8;

// BM rows of E per block, K = the contraction length (= n), WAVES waves, TN
// 16-column blocks per wave, PF steps of X loads in flight, NV vectors per
// work unit (1 for plain products, p for the squaring step's orders).
template <int BM_, int K_, int WAVES_, int TN_, int PF_, int NV_>
struct RC {
  static constexpr int BM = BM_, K = K_, WAVES = WAVES_, TN = TN_, PF = PF_, NV = NV_;
  static constexpr int NT = 64 * WAVES;
  static constexpr int RB = BM / 16;            // 16-row MFMA blocks
  static constexpr int KB = K / 64;             // 64-deep steps per vector
  static constexpr int S = NV * KB;             // steps per work unit
  static constexpr int COLS = 16 * TN * WAVES;  // output columns per work unit
  static constexpr int CHUNKS = BM * K / 4;     // 16-byte LDS chunks (hi + lo)
  static_assert(BM % 16 == 0 && K % 64 == 0, "shape");
  static_assert(PF >= 1 && PF <= S && S % PF == 0, "the load ring must tile a work unit");
};

// LDS chunk of the A fragment (row block rb, step kb, MFMA step s, plane pl)
template <class C>
__device__ __forceinline__ int frag(int rb, int kb, int s, int pl) {
  return (((rb * C::KB + kb) * 2 + s) * 2 + pl) * 64;
}

// rows row0 .. row0 + BM - 1 of E (hi, lo planes, row-major K) into LDS
template <class C>
__device__ __forceinline__ void load_e(bf8* __restrict__ els, const __bf16* __restrict__ Ehi,
                                       const __bf16* __restrict__ Elo, int row0) {
  for (int c = threadIdx.x; c < C::CHUNKS; c += C::NT) {
    const int lane = c & 63;
    int f = c >> 6;
    const int pl = f & 1;
    f >>= 1;
    const int s = f & 1;
    f >>= 1;
    const int kb = f % C::KB, rb = f / C::KB;
    const int row = row0 + rb * 16 + (lane & 15);
    const int k = kb * 64 + 16 * (lane >> 4) + 8 * s;
    els[c] = *(const bf8*)((pl ? Elo : Ehi) + (long long)row * C::K + k);
  }
}

template <class T>
struct Ring16 {
  T v[16];
};

__device__ __forceinline__ void ld16(const float* __restrict__ p, Ring16<float>& r) {
#pragma unroll
  for (int i = 0; i < 4; ++i) {
    const f4 x = *(const f4*)(p + 4 * i);
    r.v[4 * i] = x.x;
    r.v[4 * i + 1] = x.y;
    r.v[4 * i + 2] = x.z;
    r.v[4 * i + 3] = x.w;
  }
}
__device__ __forceinline__ void ld16(const double* __restrict__ p, Ring16<double>& r) {
#pragma unroll
  for (int i = 0; i < 8; ++i) {
    const dv2 x = *(const dv2*)(p + 2 * i);
    r.v[2 * i] = x.x;
    r.v[2 * i + 1] = x.y;
  }
}

// hi/lo split of elements 8 s .. 8 s + 7 (the same roundings as the general kernel)
__device__ __forceinline__ void split8(const Ring16<float>& r, int s, bf8& hi, bf8& lo) {
#pragma unroll
  for (int j = 0; j < 8; ++j) {
    const float x = r.v[8 * s + j];
    const __bf16 hb = (__bf16)x;
    hi[j] = hb;
    lo[j] = (__bf16)(x - (float)hb);
  }
}
__device__ __forceinline__ void split8(const Ring16<double>& r, int s, bf8& hi, bf8& lo) {
#pragma unroll
  for (int j = 0; j < 8; ++j) {
    const double x = r.v[8 * s + j];
    const __bf16 hb = (__bf16)(float)x;
    hi[j] = hb;
    lo[j] = (__bf16)(float)(x - (double)(float)hb);
  }
}

// a.L as a value the compiler cannot hoist products of out of the unit loop
// (it would keep one 64-bit row offset per output row in registers)
__device__ __forceinline__ long long opaque_len(int L) {
  asm volatile("" : "+s"(L));
  return (long long)L;
}

// Work assignment of one block: its row half, and its range of units
// [u0, u1) with unit u = (b = u / CT, column tile u % CT).
struct Work {
  int h;
  long long u0, u1;
  int CT;
};

template <class C>
__device__ __forceinline__ Work block_work(int M, int L, int nfac) {
  const int H = M / C::BM;
  Work w;
  const int k = blockIdx.x;
  const int x = k % kXcd, r = k / kXcd;
  w.h = r % H;
  const int q = r / H;
  const int pairs = gridDim.x / H;  // grid is a multiple of kXcd * H
  const int P = q * kXcd + x;
  w.CT = (L + C::COLS - 1) / C::COLS;
  const long long U = (long long)nfac * w.CT;
  w.u0 = U * P / pairs;
  w.u1 = U * (P + 1) / pairs;
  return w;
}

// load step t (0 <= t < S) of unit u into a ring slot
template <class C, class TIn>
__device__ __forceinline__ void load_step(const TIn* __restrict__ X, long long xs, int L, const Work& w,
                                          long long u, int t, bool per_vector, Ring16<TIn> (&slot)[C::TN]) {
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int v = t / C::KB, kb = t % C::KB;
  const int b = (int)(u / w.CT), ct = (int)(u % w.CT);
  const TIn* Xb = X + (per_vector ? (long long)v : (long long)b) * xs;
  const int k = kb * 64 + 16 * (lane >> 4);
#pragma unroll
  for (int c = 0; c < C::TN; ++c) {
    int j = ct * C::COLS + (wave * C::TN + c) * 16 + (lane & 15);
    j = j < L ? j : L - 1;
    ld16(Xb + (long long)j * C::K + k, slot[c]);
  }
}

// acc[rb][c] += A(rb, kb) B(c) for both MFMA steps of one 64-deep step.
// The A fragments of row block rb + 1 are read while rb's products run; the
// scheduling barriers keep the compiler from hoisting every read of the step
// (which would hold 32 fragments, 128 registers, at once).
template <class C, class TIn>
__device__ __forceinline__ void mma_step(const bf8* __restrict__ els, int kb, const Ring16<TIn> (&slot)[C::TN],
                                         f4 (&acc)[C::RB][C::TN]) {
  const int lane = threadIdx.x & 63;
#pragma unroll
  for (int s = 0; s < 2; ++s) {
    bf8 bh[C::TN], bl[C::TN];
#pragma unroll
    for (int c = 0; c < C::TN; ++c) split8(slot[c], s, bh[c], bl[c]);
    bf8 ah = els[frag<C>(0, kb, s, 0) + lane];
    bf8 al = els[frag<C>(0, kb, s, 1) + lane];
#pragma unroll
    for (int rb = 0; rb < C::RB; ++rb) {
      bf8 nh, nl;
      if (rb + 1 < C::RB) {
        nh = els[frag<C>(rb + 1, kb, s, 0) + lane];
        nl = els[frag<C>(rb + 1, kb, s, 1) + lane];
      }
#pragma unroll
      for (int c = 0; c < C::TN; ++c) {
        acc[rb][c] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(al, bh[c], acc[rb][c], 0, 0, 0);
        acc[rb][c] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(ah, bl[c], acc[rb][c], 0, 0, 0);
        acc[rb][c] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(ah, bh[c], acc[rb][c], 0, 0, 0);
      }
      __builtin_amdgcn_sched_barrier(0);
      if (rb + 1 < C::RB) {
        ah = nh;
        al = nl;
      }
    }
  }
}

// The shared driver: E reloads, the load ring across units, the MFMA steps;
// epi(u, acc) is called once per unit with the NV accumulator sets.
template <class C, class TIn, class Epi>
__device__ __forceinline__ void run_units(const TtmArgs& a, bool per_vector, int nfac, bf8* __restrict__ els,
                                          Epi&& epi) {
  const Work w = block_work<C>(a.M, a.L, nfac);
  if (w.u0 >= w.u1) return;
  const TIn* X = (const TIn*)a.X;
  const __bf16* Ehi = (const __bf16*)a.Ea;
  const __bf16* Elo = (const __bf16*)a.Eb;
  Ring16<TIn> ring[C::PF][C::TN];
  // prologue: the first PF steps (PF <= S: all in the first unit)
#pragma unroll
  for (int t = 0; t < C::PF; ++t) load_step<C, TIn>(X, a.xs, a.L, w, w.u0, t, per_vector, ring[t]);
  int loaded = -1;
  for (long long u = w.u0; u < w.u1; ++u) {
    const int b = (int)(u / w.CT);
    const int fac = a.es == 0 ? 0 : b;
    if (fac != loaded) {
      __syncthreads();  // every wave is done with the previous factor
      load_e<C>(els, Ehi + (long long)fac * a.es, Elo + (long long)fac * a.es, w.h * C::BM);
      __syncthreads();
      loaded = fac;
    }
    f4 acc[C::NV][C::RB][C::TN];
#pragma unroll
    for (int v = 0; v < C::NV; ++v)
#pragma unroll
      for (int rb = 0; rb < C::RB; ++rb)
#pragma unroll
        for (int c = 0; c < C::TN; ++c) acc[v][rb][c] = (f4){0.f, 0.f, 0.f, 0.f};
#pragma unroll
    for (int t = 0; t < C::S; ++t) {
      // the factor's fragments are the same for every vector of a unit: keep
      // the compiler from holding them all in registers across vectors
      asm volatile("" ::: "memory");
      const int slot = t % C::PF;
      Ring16<TIn> cur[C::TN];
#pragma unroll
      for (int c = 0; c < C::TN; ++c) cur[c] = ring[slot][c];
      // refill the slot with the step PF ahead (maybe in the next unit)
      const int tn = t + C::PF;
      if (tn < C::S)
        load_step<C, TIn>(X, a.xs, a.L, w, u, tn, per_vector, ring[slot]);
      else if (u + 1 < w.u1)
        load_step<C, TIn>(X, a.xs, a.L, w, u + 1, tn - C::S, per_vector, ring[slot]);
      mma_step<C, TIn>(els, t % C::KB, cur, acc[t / C::KB]);
    }
    epi(u, w, acc);
  }
}

template <class C, class TIn, class TOut>
__global__ __launch_bounds__(C::NT) void ttm_bf16r_store_kernel(TtmArgs a) {
  __shared__ bf8 els[C::CHUNKS];
  if (a.stop && *a.stop) return;
  run_units<C, TIn>(a, false, a.nbatch, els, [&](long long u, const Work& w, f4 (&acc)[C::NV][C::RB][C::TN]) {
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int b = (int)(u / w.CT), ct = (int)(u % w.CT);
    TOut* O = (TOut*)a.O + (long long)b * a.os;
    const long long L = opaque_len(a.L);
#pragma unroll
    for (int c = 0; c < C::TN; ++c) {
      const int col = ct * C::COLS + (wave * C::TN + c) * 16 + (lane & 15);
      if (col >= a.L) continue;
#pragma unroll
      for (int rb = 0; rb < C::RB; ++rb)
#pragma unroll
        for (int e = 0; e < 4; ++e) {
          const int row = w.h * C::BM + rb * 16 + 4 * (lane >> 4) + e;
          O[row * L + col] = (TOut)acc[0][rb][c][e];
        }
    }
  });
}

// Squaring step, all NV = p orders per block (eq. squaring):
// O_i = 2^{-i} (E X_i + sum_{j=1}^{i} Y_j / (i-j)!), i = 1..p, Y_j read once.
template <class C, class TIn>
__global__ __launch_bounds__(C::NT) void ttm_bf16r_square_kernel(TtmArgs a) {
  __shared__ bf8 els[C::CHUNKS];
  run_units<C, TIn>(a, true, 1, els, [&](long long u, const Work& w, f4 (&acc)[C::NV][C::RB][C::TN]) {
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int ct = (int)(u % w.CT);
    const long long L = opaque_len(a.L);
#pragma unroll
    for (int c = 0; c < C::TN; ++c) {
      const int col = ct * C::COLS + (wave * C::TN + c) * 16 + (lane & 15);
      if (col >= a.L) continue;
#pragma unroll
      for (int rb = 0; rb < C::RB; ++rb)
#pragma unroll
        for (int e = 0; e < 4; ++e) {
          const int row = w.h * C::BM + rb * 16 + 4 * (lane >> 4) + e;
          const long long idx = row * L + col;
          double y[C::NV];
#pragma unroll
          for (int j = 0; j < C::NV; ++j) y[j] = a.Yprev[j * a.yps + idx];
#pragma unroll
          for (int i = 0; i < C::NV; ++i) {
            double s = (double)acc[i][rb][c][e];
#pragma unroll
            for (int j = 0; j <= i; ++j) s += y[j] * a.ifact[i - j];
            ((double*)a.O)[i * a.os + idx] = ldexp(1.0, -(i + 1)) * s;
          }
          // keep the loads of the next element group behind this one: hoisting
          // them all would hold every y_j of the tile in registers
          __builtin_amdgcn_sched_barrier(0);
        }
    }
  });
}

inline int cu_count() {
  static int n = 0;
  if (!n) {
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess ||
        hipDeviceGetAttribute(&n, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess || n <= 0)
      n = 256;
  }
  return n;
}

// Persistent grid: co-resident blocks, a multiple of kXcd * (row halves).
template <class C, class F>
int grid_of(F kernel, int M) {
  static int per_cu = 0;
  if (!per_cu) {
    int b = 0;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&b, kernel, C::NT, 0) != hipSuccess || b < 1) b = 1;
    per_cu = b;
  }
  const int H = M / C::BM;
  int g = cu_count() * per_cu;
  g = (g / (kXcd * H)) * (kXcd * H);
  return g < kXcd * H ? kXcd * H : g;
}

template <class C, class TIn, class TOut>
int store_go(const TtmArgs& a, hipStream_t st) {
  auto k = ttm_bf16r_store_kernel<C, TIn, TOut>;
  const int g = grid_of<C>(k, a.M);
  PHIQ_LAUNCH_R(k, dim3(g), dim3(C::NT), 0, st, a);
  return hipGetLastError();
}

// FP64 inputs (the squaring iterates, phi_0's input) take half the ring:
// 16 doubles per column block and step are 32 registers
template <template <class> class Sel>
int by_types(const TtmArgs& a, hipStream_t st) {
  if (a.x_f32 && a.o_f32) return store_go<typename Sel<float>::C, float, float>(a, st);
  if (a.x_f32) return store_go<typename Sel<float>::C, float, double>(a, st);
  if (a.o_f32) return store_go<typename Sel<double>::C, double, float>(a, st);
  return store_go<typename Sel<double>::C, double, double>(a, st);
}

template <int BM, int K, int WAVES, int TN, int PF32>
struct StoreSel {
  template <class TIn>
  struct T {
    static constexpr int PF = sizeof(TIn) == 8 ? (PF32 >= 2 ? PF32 / 2 : 1) : PF32;
    using C = RC<BM, K, WAVES, TN, PF, 1>;
  };
};

template <class C, class TIn>
int square_go(const TtmArgs& a, hipStream_t st) {
  auto k = ttm_bf16r_square_kernel<C, TIn>;
  const int g = grid_of<C>(k, a.M);
  PHIQ_LAUNCH_R(k, dim3(g), dim3(C::NT), 0, st, a);
  return hipGetLastError();
}

template <int BM, int K, int NV, int WAVES>
int square_np(const TtmArgs& a, hipStream_t st) {
  // p accumulator sets per wave: one 16-column block per wave and a ring of
  // two steps keep them in registers
  constexpr int S = NV * (K / 64);
  using C = RC<BM, K, WAVES, 1, (S % 2 == 0 ? 2 : 1), NV>;
  return a.x_f32 ? square_go<C, float>(a, st) : square_go<C, double>(a, st);
}

template <int BM, int K, int WAVES>
int square_waves(const TtmArgs& a, hipStream_t st) {
  switch (a.nbatch) {
    case 1: return square_np<BM, K, 1, WAVES>(a, st);
    case 2: return square_np<BM, K, 2, WAVES>(a, st);
    case 3: return square_np<BM, K, 3, WAVES>(a, st);
    default: return square_np<BM, K, 4, WAVES>(a, st);
  }
}

template <int BM, int K>
int square_shape(const TtmArgs& a, hipStream_t st, int cfg) {
  return cfg == 2 ? square_waves<BM, K, 12>(a, st) : square_waves<BM, K, 8>(a, st);
}

template <int BM, int K>
int store_shape(const TtmArgs& a, hipStream_t st, int cfg) {
  constexpr int KB = K / 64;
  switch (cfg) {
    case 2: return by_types<StoreSel<BM, K, 4, 2, KB>::template T>(a, st);
    case 3: return by_types<StoreSel<BM, K, 8, 2, (KB >= 2 ? 2 : 1)>::template T>(a, st);
    case 4: return by_types<StoreSel<BM, K, 12, 1, (KB >= 2 ? 2 : 1)>::template T>(a, st);
    case 5: return by_types<StoreSel<BM, K, 16, 1, (KB >= 2 ? 2 : 1)>::template T>(a, st);
    case 1: return by_types<StoreSel<BM, K, 8, 1, KB>::template T>(a, st);
    default: return by_types<StoreSel<BM, K, 16, 1, (KB >= 2 ? 2 : 1)>::template T>(a, st);
  }
}

// shapes the resident kernels take: M = K = n in {64, 128, 256}, 16-byte
// aligned operands, one batch stride per factor
bool bf16r_shape(const TtmArgs& a) {
  if (a.nn || a.M != a.K || !(a.K == 64 || a.K == 128 || a.K == 256)) return false;
  if (!a.Ea || !a.Eb || a.L < 1) return false;
  if (((uintptr_t)a.Ea | (uintptr_t)a.Eb | (uintptr_t)a.X) % 16 != 0) return false;
  if (a.es % 8 != 0 || a.xs % 8 != 0) return false;
  return true;
}

}  // namespace

int bf16r_num_configs() { return 6; }
int bf16r_square_num_configs() { return 3; }

// cfg: 0 = decline (the caller runs the general kernel), 1..5 resident
// shapes (1: eight waves of 16 columns, 2: four waves of 32, 3: eight waves
// of 32, 4: twelve waves of 16, 5: sixteen waves of 16), -1 = default (5:
// at n = 256 and 128 it measured best, by 2%).
// Squaring: 1 eight waves, 2 twelve waves.  Returns hipErrorNotSupported for shapes the
// resident kernels do not take.
int launch_ttm_store_bf16r(const TtmArgs& a, void* stream, int cfg) {
  if (cfg == 0 || !bf16r_shape(a) || a.nbatch < 1) return hipErrorNotSupported;
  // by default only launches with enough 128-column units to fill the GPU
  const long long units = (long long)a.nbatch * ((a.L + 127) / 128) * (a.M / (a.K == 64 ? 64 : 128));
  if (cfg < 0 && units < cu_count()) return hipErrorNotSupported;
  hipStream_t st = (hipStream_t)stream;
  if (a.K == 256) return store_shape<128, 256>(a, st, cfg);
  if (a.K == 128) return store_shape<128, 128>(a, st, cfg);
  return store_shape<64, 64>(a, st, cfg);
}

int launch_ttm_square_bf16r(const TtmArgs& a, void* stream, int cfg) {
  if (cfg == 0 || !bf16r_shape(a) || a.nbatch < 1 || a.nbatch > 4 || a.es != 0 || a.order0 != 0 || a.yacc ||
      a.yps % 2 != 0)
    return hipErrorNotSupported;
  const long long units = (long long)((a.L + 127) / 128) * (a.M / (a.K == 64 ? 64 : 128));
  if (cfg < 0 && units < cu_count()) return hipErrorNotSupported;
  hipStream_t st = (hipStream_t)stream;
  if (a.K == 256) return square_shape<128, 256>(a, st, cfg);
  if (a.K == 128) return square_shape<128, 128>(a, st, cfg);
  return square_shape<64, 64>(a, st, cfg);
}

}  // namespace phiq
