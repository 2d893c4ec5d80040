// FP32 mode products with the 1D factor resident in LDS (gfx950), the FP32
// form of the resident-factor FP64 kernels (kernels_f64r.hip):
//
//   out[i][j] = sum_k E[i][k] X[j][k],  i < M = K = n,  j < L,
//
// on v_mfma_f32_16x16x4_f32 with the FP32 copy of E (the plan's twin) and
// FP32 or FP64 X, for n in {128, 256}: the plain product (Kronecker chains;
// FP32 or FP64 output) and the product fused with the modified squaring of
// eq. squaring (FP64 iterates and output).
//   * A block keeps BM rows of E (BM x K floats: 128 KB at n = 256 with half
//     the rows, 64 KB at n = 128 with all of them) in LDS for as long as it
//     works with that factor, in MFMA fragment order: a lane's four operands
//     of four MFMAs are one 16-byte read.
//   * Waves stream X straight into registers: a wave owns 16 TN columns of
//     the output and RB row blocks; it walks K in 32-deep steps, each lane
//     loading 8 consecutive k of one column, PF steps of loads in flight
//     across unit boundaries.  No barrier in the steady state.
//   * Inside a 32-deep step the k order is permuted in both operands alike:
//     lane group g (= lane / 16) of MFMA s (0..7) covers k = 8 g + s.  The
//     sum over k is unchanged; its rounding order differs from the general
//     FP32 kernel's.
//   * Persistent blocks take contiguous ranges of work units (factor b, row
//     part h, column tile), factor-major; the H row parts of a column tile
//     run on one XCD (block ids k, k + 8, ...), so the second read of an X
//     strip can come from that XCD's L2.
// The FP32 MFMA's output layout differs from the FP64 one: lane l, element
// e holds D[4 (l / 16) + e][l % 16].
#include <hip/hip_ext.h>
#include <hip/hip_runtime.h>

#include "phiq_internal.h"

namespace phiq {

#define PHIQ_LAUNCH_G(K, G, B, SH, ST, ...)                                                               \
  do {                                                                                                    \
    if (g_launch_events[0])                                                                               \
      hipExtLaunchKernelGGL(K, G, B, SH, ST, (hipEvent_t)g_launch_events[0], (hipEvent_t)g_launch_events[1], \
                            0, __VA_ARGS__);                                                              \
    else                                                                                                  \
      hipLaunchKernelGGL(K, G, B, SH, ST, __VA_ARGS__);                                                   \
  } while (0)

namespace {

typedef float fq __attribute__((ext_vector_type(4)));
typedef double dp2 __attribute__((ext_vector_type(2)));

constexpr int kXcdG = 8;

// BM rows of E per block, K = n, WR x WC waves (row groups x column
// groups), TN 16-column blocks per wave, PF steps of loads in flight, NV
// vectors per work unit (1 for plain products, the orders of a squaring step).
template <int BM_, int K_, int WR_, int WC_, int TN_, int PF_, int NV_>
struct GC {
  static constexpr int BM = BM_, K = K_, WR = WR_, WC = WC_, TN = TN_, PF = PF_, NV = NV_;
  static constexpr int WAVES = WR * WC;
  static constexpr int NT = 64 * WAVES;
  static constexpr int RB = BM / 16 / WR;       // 16-row blocks per wave
  static constexpr int KB = K / 32;             // 32-deep steps per vector
  static constexpr int S = NV * KB;             // steps per work unit
  static constexpr int COLS = 16 * TN * WC;     // output columns per work unit
  static constexpr int QUADS = BM * K / 4;      // 16-byte LDS entries
  static_assert(BM % (16 * WR) == 0 && K % 32 == 0, "shape");
  static_assert(PF >= 1 && PF <= S && S % PF == 0, "the load ring must tile a work unit");
};

// LDS entry of the operand quad q (k = 8 g + 4 q .. + 3) of row block rb
// (within the block's BM rows) and step kb, for lane 0
template <class C>
__device__ __forceinline__ int frag(int rb, int kb, int q) {
  return ((rb * C::KB + kb) * 2 + q) * 64;
}

// rows row0 .. row0 + BM - 1 of E (row-major FP32, K columns) into LDS
template <class C>
__device__ __forceinline__ void load_e(fq* __restrict__ els, const float* __restrict__ E, int row0) {
#pragma unroll 4
  for (int c = threadIdx.x; c < C::QUADS; c += C::NT) {
    const int lane = c & 63;
    int f = c >> 6;
    const int q = f & 1;
    f >>= 1;
    const int kb = f % C::KB, rb = f / C::KB;
    const int row = row0 + rb * 16 + (lane & 15);
    const int k = kb * 32 + 8 * (lane >> 4) + 4 * q;
    els[c] = *(const fq*)(E + (long long)row * C::K + k);
  }
}

struct Ring8f {
  float v[8];
};

__device__ __forceinline__ void ld8(const float* __restrict__ p, Ring8f& r) {
#pragma unroll
  for (int i = 0; i < 2; ++i) {
    const fq x = *(const fq*)(p + 4 * i);
    r.v[4 * i] = x.x;
    r.v[4 * i + 1] = x.y;
    r.v[4 * i + 2] = x.z;
    r.v[4 * i + 3] = x.w;
  }
}
// FP64 input (the first product of a chain): rounded to FP32 as it arrives,
// as the general FP32 kernel rounds it at its staging
__device__ __forceinline__ void ld8(const double* __restrict__ p, Ring8f& r) {
#pragma unroll
  for (int i = 0; i < 4; ++i) {
    const dp2 x = *(const dp2*)(p + 2 * i);
    r.v[2 * i] = (float)x.x;
    r.v[2 * i + 1] = (float)x.y;
  }
}

// a.L as a value the compiler cannot hoist products of out of the unit loop
__device__ __forceinline__ long long opaque_len_g(int L) {
  asm volatile("" : "+s"(L));
  return (long long)L;
}

struct WorkG {
  int h;
  long long u0, u1;
  int CT;
};

template <class C>
__device__ __forceinline__ WorkG block_work(int M, int L, int nfac) {
  const int H = M / C::BM;
  WorkG w;
  const int k = blockIdx.x;
  const int x = k % kXcdG, r = k / kXcdG;
  w.h = r % H;
  const int q = r / H;
  const int groups = gridDim.x / H;  // grid is a multiple of kXcdG * H
  const int P = q * kXcdG + x;
  w.CT = (L + C::COLS - 1) / C::COLS;
  const long long U = (long long)nfac * w.CT;
  w.u0 = U * P / groups;
  w.u1 = U * (P + 1) / groups;
  return w;
}

// load step t (0 <= t < S) of unit u into a ring slot
template <class C, class TIn>
__device__ __forceinline__ void load_step(const TIn* __restrict__ X, long long xs, int L, const WorkG& w,
                                          long long u, int t, bool per_vector, Ring8f (&slot)[C::TN]) {
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int wc = wave % C::WC;
  const int v = t / C::KB, kb = t % C::KB;
  const int b = (int)(u / w.CT), ct = (int)(u % w.CT);
  const TIn* Xb = X + (per_vector ? (long long)v : (long long)b) * xs;
  const int k = kb * 32 + 8 * (lane >> 4);
#pragma unroll
  for (int c = 0; c < C::TN; ++c) {
    int j = ct * C::COLS + (wc * C::TN + c) * 16 + (lane & 15);
    j = j < L ? j : L - 1;
    ld8(Xb + (long long)j * C::K + k, slot[c]);
  }
}

// acc[rb][c] += A(rb, kb) B(c): the eight MFMAs of one 32-deep step per
// (row block, column block).  The A quads of the second half are read while
// the first half's products run.
template <class C>
__device__ __forceinline__ void mma_step(const fq* __restrict__ els, int kb, const Ring8f (&b)[C::TN],
                                         fq (&acc)[C::RB][C::TN]) {
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int rb0 = (wave / C::WC) * C::RB;
  fq a[C::RB];
#pragma unroll
  for (int rb = 0; rb < C::RB; ++rb) a[rb] = els[frag<C>(rb0 + rb, kb, 0) + lane];
#pragma unroll
  for (int q = 0; q < 2; ++q) {
    fq n[C::RB];
    if (q == 0) {
#pragma unroll
      for (int rb = 0; rb < C::RB; ++rb) n[rb] = els[frag<C>(rb0 + rb, kb, 1) + lane];
    }
#pragma unroll
    for (int s = 0; s < 4; ++s)
#pragma unroll
      for (int rb = 0; rb < C::RB; ++rb)
#pragma unroll
        for (int c = 0; c < C::TN; ++c)
          acc[rb][c] = __builtin_amdgcn_mfma_f32_16x16x4f32(a[rb][s], b[c].v[4 * q + s], acc[rb][c], 0, 0, 0);
    __builtin_amdgcn_sched_barrier(0);
    if (q == 0) {
#pragma unroll
      for (int rb = 0; rb < C::RB; ++rb) a[rb] = n[rb];
    }
  }
}

// The shared driver: E reloads, the load ring across units, the MFMA steps;
// epi(u, w, acc) runs once per unit with the NV accumulator sets.
template <class C, class TIn, class Epi>
__device__ __forceinline__ void run_units(const TtmArgs& a, bool per_vector, int nfac, fq* __restrict__ els,
                                          Epi&& epi) {
  const WorkG w = block_work<C>(a.M, a.L, nfac);
  if (w.u0 >= w.u1) return;
  const TIn* X = (const TIn*)a.X;
  const float* E = (const float*)a.Ea;
  Ring8f ring[C::PF][C::TN];
#pragma unroll
  for (int t = 0; t < C::PF; ++t) load_step<C, TIn>(X, a.xs, a.L, w, w.u0, t, per_vector, ring[t]);
  int loaded = -1;
  for (long long u = w.u0; u < w.u1; ++u) {
    const int b = (int)(u / w.CT);
    const int fac = a.es == 0 ? 0 : b;
    if (fac != loaded) {
      __syncthreads();  // every wave is done with the previous factor
      load_e<C>(els, E + (long long)fac * a.es, w.h * C::BM);
      __syncthreads();
      loaded = fac;
    }
    fq acc[C::NV][C::RB][C::TN];
#pragma unroll
    for (int v = 0; v < C::NV; ++v)
#pragma unroll
      for (int rb = 0; rb < C::RB; ++rb)
#pragma unroll
        for (int c = 0; c < C::TN; ++c) acc[v][rb][c] = (fq){0.f, 0.f, 0.f, 0.f};
#pragma unroll
    for (int t = 0; t < C::S; ++t) {
      // the factor's quads are the same for every vector of a unit: keep the
      // compiler from holding them all in registers across vectors
      asm volatile("" ::: "memory");
      const int slot = t % C::PF;
      Ring8f cur[C::TN];
#pragma unroll
      for (int c = 0; c < C::TN; ++c) cur[c] = ring[slot][c];
      const int tn = t + C::PF;
      if (tn < C::S)
        load_step<C, TIn>(X, a.xs, a.L, w, u, tn, per_vector, ring[slot]);
      else if (u + 1 < w.u1)
        load_step<C, TIn>(X, a.xs, a.L, w, u + 1, tn - C::S, per_vector, ring[slot]);
      mma_step<C>(els, t % C::KB, cur, acc[t / C::KB]);
    }
    epi(u, w, acc);
  }
}

// output row and column of accumulator element e of (row block rb, column
// block c) of this lane
template <class C>
__device__ __forceinline__ int out_row(const WorkG& w, int rb, int e) {
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  return w.h * C::BM + ((wave / C::WC) * C::RB + rb) * 16 + 4 * (lane >> 4) + e;
}
template <class C>
__device__ __forceinline__ int out_col(int ct, int c) {
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  return ct * C::COLS + ((wave % C::WC) * C::TN + c) * 16 + (lane & 15);
}

template <class C, class TIn, class TOut>
__global__ __launch_bounds__(C::NT) void ttm_f32r_store_kernel(TtmArgs a) {
  __shared__ fq els[C::QUADS];
  if (a.stop && *a.stop) return;
  run_units<C, TIn>(a, false, a.nbatch, els, [&](long long u, const WorkG& w, fq (&acc)[C::NV][C::RB][C::TN]) {
    const int b = (int)(u / w.CT), ct = (int)(u % w.CT);
    TOut* O = (TOut*)a.O + (long long)b * a.os;
    const long long L = opaque_len_g(a.L);
#pragma unroll
    for (int c = 0; c < C::TN; ++c) {
      const int col = out_col<C>(ct, c);
      if (col >= a.L) continue;
#pragma unroll
      for (int rb = 0; rb < C::RB; ++rb)
#pragma unroll
        for (int e = 0; e < 4; ++e) O[out_row<C>(w, rb, e) * L + col] = (TOut)acc[0][rb][c][e];
    }
  });
}

// Squaring step (eq. squaring), NV orders per block: batch i is order
// o = i + 1 + order0 and O_i = 2^{-o} (E X_i + sum_{j=1}^{o} Y_j / (o-j)!),
// added to O_i when yacc is set; the NY = order0 + NV iterates Y_j (FP64)
// are read once per element.
template <class C, int NY>
__global__ __launch_bounds__(C::NT) void ttm_f32r_square_kernel(TtmArgs a) {
  __shared__ fq els[C::QUADS];
  if (a.stop && *a.stop) return;
  run_units<C, float>(a, true, 1, els, [&](long long u, const WorkG& w, fq (&acc)[C::NV][C::RB][C::TN]) {
    const int ct = (int)(u % w.CT);
    const long long L = opaque_len_g(a.L);
#pragma unroll
    for (int c = 0; c < C::TN; ++c) {
      const int col = out_col<C>(ct, c);
      if (col >= a.L) continue;
#pragma unroll
      for (int rb = 0; rb < C::RB; ++rb)
#pragma unroll
        for (int e = 0; e < 4; ++e) {
          const long long idx = out_row<C>(w, rb, e) * L + col;
          double y[NY];
#pragma unroll
          for (int j = 0; j < NY; ++j) y[j] = a.Yprev[j * a.yps + idx];
#pragma unroll
          for (int i = 0; i < C::NV; ++i) {
            const int o = i + 1 + (NY - C::NV);
            double s = (double)acc[i][rb][c][e];
#pragma unroll
            for (int j = 0; j < o; ++j) s += y[j] * a.ifact[o - 1 - j];
            double* O = (double*)a.O + i * a.os + idx;
            const double r = ldexp(1.0, -o) * s;
            *O = a.yacc ? *O + r : r;
          }
          // keep the next element group's loads behind this one
          __builtin_amdgcn_sched_barrier(0);
        }
    }
  });
}

inline int cu_count_g() {
  static int n = 0;
  if (!n) {
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess ||
        hipDeviceGetAttribute(&n, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess || n <= 0)
      n = 256;
  }
  return n;
}

// Persistent grid: co-resident blocks, a multiple of kXcdG * (row parts),
// at most one block per unit group.  per_cu caches the kernel's occupancy
// (one per instantiation: variants of one shape differ in registers).
template <class C, class F>
int grid_of(F kernel, int& per_cu, int M, long long units) {
  if (!per_cu) {
    int b = 0;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&b, kernel, C::NT, 0) != hipSuccess || b < 1) b = 1;
    per_cu = b;
  }
  const int H = M / C::BM;
  long long g = (long long)cu_count_g() * per_cu;
  g = std::min<long long>(g, units * H);
  g = (g / (kXcdG * H)) * (kXcdG * H);
  return (int)(g < kXcdG * H ? kXcdG * H : g);
}

template <class C, class TIn, class TOut>
int store_go(const TtmArgs& a, hipStream_t st) {
  static int per_cu = 0;
  auto k = ttm_f32r_store_kernel<C, TIn, TOut>;
  const long long units = (long long)a.nbatch * ((a.L + C::COLS - 1) / C::COLS);
  const int g = grid_of<C>(k, per_cu, a.M, units);
  PHIQ_LAUNCH_G(k, dim3(g), dim3(C::NT), 0, st, a);
  return hipGetLastError();
}

template <class C>
int store_io(const TtmArgs& a, hipStream_t st) {
  if (a.x_f32) return a.o_f32 ? store_go<C, float, float>(a, st) : store_go<C, float, double>(a, st);
  return a.o_f32 ? store_go<C, double, float>(a, st) : store_go<C, double, double>(a, st);
}

// cfg 1: 128 rows per block (all rows at n = 128, half at n = 256), eight
// waves side by side (128-column units); cfg 2: sixteen waves (256-column
// units); cfg 3: 64 rows per block, eight waves.
template <int K>
int store_shape(const TtmArgs& a, hipStream_t st, int cfg) {
  constexpr int PF8 = (K / 32 >= 4 ? 4 : K / 32), PF16 = (K / 32 >= 2 ? 2 : 1);
  if (cfg == 2) return store_io<GC<128, K, 1, 16, 1, PF16, 1>>(a, st);
  if (cfg == 3) return store_io<GC<64, K, 1, 8, 1, PF8, 1>>(a, st);
  return store_io<GC<128, K, 1, 8, 1, PF8, 1>>(a, st);
}

template <class C, int NY>
int square_go(const TtmArgs& a, hipStream_t st) {
  static int per_cu = 0;
  auto k = ttm_f32r_square_kernel<C, NY>;
  const long long units = (a.L + C::COLS - 1) / C::COLS;
  const int g = grid_of<C>(k, per_cu, a.M, units);
  PHIQ_LAUNCH_G(k, dim3(g), dim3(C::NT), 0, st, a);
  return hipGetLastError();
}

template <int K, int NV, int BM, int WC>
int square_nv(const TtmArgs& a, hipStream_t st) {
  constexpr int S = NV * (K / 32);
  using C = GC<BM, K, 1, WC, 1, (S % 4 == 0 ? 4 : (S % 2 == 0 ? 2 : 1)), NV>;
  switch (a.order0 + NV) {
    case 1: return square_go<C, (NV <= 1 ? 1 : NV)>(a, st);
    case 2: return square_go<C, (NV <= 2 ? 2 : NV)>(a, st);
    case 3: return square_go<C, (NV <= 3 ? 3 : NV)>(a, st);
    default: return square_go<C, 4>(a, st);
  }
}

template <int K, int BM, int WC>
int square_shape(const TtmArgs& a, hipStream_t st) {
  switch (a.nbatch) {
    case 1: return square_nv<K, 1, BM, WC>(a, st);
    case 2: return square_nv<K, 2, BM, WC>(a, st);
    case 3: return square_nv<K, 3, BM, WC>(a, st);
    default: return square_nv<K, 4, BM, WC>(a, st);
  }
}

// launches the resident kernels take: the FP32 twin of E, FP32 or FP64 X,
// rotated layout, M = K = n in {128, 256}, 16-byte aligned operands, one
// batch stride per factor, no two-index batches
bool f32r_shape(const TtmArgs& a) {
  if (a.nn || !a.Ea || a.M != a.K || !(a.K == 128 || a.K == 256)) return false;
  if (a.emod > 0 || a.xdiv > 0 || a.nouter > 1 || a.seg.n > 0 || a.L < 1 || a.nbatch < 1) return false;
  if (((uintptr_t)a.Ea | (uintptr_t)a.X) % 16 != 0) return false;
  if (a.es % 4 != 0 || a.xs % 4 != 0) return false;
  return true;
}

}  // namespace

// FP32 plain products.  cfg: 0 = decline (the caller runs the general FP32
// kernel), 1..3 the shapes of store_shape, -1 = default (cfg 1 at n = 256
// when there is at least one unit per CU, else decline: at n = 128 the
// general kernel measured faster).  Returns hipErrorNotSupported for
// launches these kernels do not take.
int launch_ttm_store_f32r(const TtmArgs& a, void* stream, int cfg) {
  if (cfg == 0 || cfg > 3 || !f32r_shape(a)) return hipErrorNotSupported;
  if (cfg < 0) {
    const long long units = (long long)a.nbatch * ((a.L + 127) / 128) * 2;
    if (a.K != 256 || units < cu_count_g()) return hipErrorNotSupported;
    cfg = 1;
  }
  hipStream_t st = (hipStream_t)stream;
  if (a.K == 256) return store_shape<256>(a, st, cfg);
  return store_shape<128>(a, st, cfg);
}

// FP32 squaring products (FP32 X, FP64 iterates and output): cfg 1 = 64 rows
// per block, eight waves side by side (128-column units), 2 = 64 rows, four
// waves, 0 = decline, -1 = default (cfg 1 when there is at least one unit
// per CU).
int launch_ttm_square_f32r(const TtmArgs& a, void* stream, int cfg) {
  if (cfg == 0 || cfg > 2 || !f32r_shape(a) || !a.x_f32 || a.nbatch > 4 || a.es != 0 || a.order0 < 0 ||
      a.order0 + a.nbatch > 4 || a.yps % 2 != 0 || (a.nbatch > 1 && a.os % 2 != 0))
    return hipErrorNotSupported;
  if (cfg < 0) {
    const long long units = (long long)((a.L + 127) / 128) * (a.K / 64);
    if (units < cu_count_g()) return hipErrorNotSupported;
    cfg = 1;
  }
  hipStream_t st = (hipStream_t)stream;
  if (cfg == 2) return a.K == 256 ? square_shape<256, 64, 4>(a, st) : square_shape<128, 64, 4>(a, st);
  return a.K == 256 ? square_shape<256, 64, 8>(a, st) : square_shape<128, 64, 8>(a, st);
}

}  // namespace phiq
