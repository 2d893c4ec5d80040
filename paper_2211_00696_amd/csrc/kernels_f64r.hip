// FP64 mode products with the 1D factor resident in LDS (gfx950).
//
//   out[i][j] = sum_k E[i][k] X[j][k],  i < M = K = n,  j < L,
//
// on v_mfma_f64_16x16x4_f64, for n in {64, 128, 256}: the plain product
// (Kronecker chains) and the product fused with the modified squaring of
// eq. squaring.  The tile kernels (kernels.hip) stage a panel of E and of X
// through LDS per 16- or 32-deep chunk with a barrier each time; with K = 128
// a tile runs four or eight chunks, so a single-vector product (512 tiles,
// two per CU) spends as long filling and draining the pipeline as in the
// matrix pipe.  Here:
//   * A block keeps BM rows of E (BM x K doubles: 128 KB at n = 128 with all
//     rows, at n = 256 with a quarter of them) in LDS for as long as it works
//     with that factor, in MFMA fragment order (a lane's pair of operands is
//     one 16-byte read; consecutive lanes read consecutive 16 bytes).
//   * Waves stream X from global memory straight into registers: a wave owns
//     16 TN columns of the output and RB row blocks; it walks K in 32-deep
//     steps, each lane loading 8 consecutive k of one column (64 bytes), and
//     keeps PF steps of loads in flight across unit boundaries.  No barrier
//     in the steady state.
//   * Inside a 32-deep step the k order is permuted in both operands alike:
//     lane group g (= lane / 16) of MFMA s (0..7) covers k = 8 g + s.  The
//     sum over k is unchanged; only its rounding order differs from the tile
//     kernels'.
//   * Persistent blocks take contiguous ranges of work units (factor b, row
//     part h, column tile), factor-major.  With H row parts (n = 256: four)
//     the H blocks of a group have ids k, k + 8, ... on one XCD and take the
//     same column tiles, so repeated reads of an X tile can come from that
//     XCD's L2.
#include <hip/hip_ext.h>
#include <hip/hip_runtime.h>

#include "phiq_internal.h"

namespace phiq {

#define PHIQ_LAUNCH_F(K, G, B, SH, ST, ...)                                                               \
  do {                                                                                                    \
    if (g_launch_events[0])                                                                               \
      hipExtLaunchKernelGGL(K, G, B, SH, ST, (hipEvent_t)g_launch_events[0], (hipEvent_t)g_launch_events[1], \
                            0, __VA_ARGS__);                                                              \
    else                                                                                                  \
      hipLaunchKernelGGL(K, G, B, SH, ST, __VA_ARGS__);                                                   \
  } while (0)

namespace {

typedef double dv2 __attribute__((ext_vector_type(2)));
typedef double dacc __attribute__((ext_vector_type(4)));

constexpr int kXcd = 8;

// BM rows of E per block, K = n, WR x WC waves (row groups x column
// groups), TN 16-column blocks per wave, PF steps of loads in flight, NV
// vectors per work unit (1 for plain products, the orders of a squaring
// step), NY previous iterates read by the squaring epilogue.
template <int BM_, int K_, int WR_, int WC_, int TN_, int PF_, int NV_>
struct FC {
  static constexpr int BM = BM_, K = K_, WR = WR_, WC = WC_, TN = TN_, PF = PF_, NV = NV_;
  static constexpr int WAVES = WR * WC;
  static constexpr int NT = 64 * WAVES;
  static constexpr int RB = BM / 16 / WR;       // 16-row blocks per wave
  static constexpr int KB = K / 32;             // 32-deep steps per vector
  static constexpr int S = NV * KB;             // steps per work unit
  static constexpr int COLS = 16 * TN * WC;     // output columns per work unit
  static constexpr int PAIRS = BM * K / 2;      // 16-byte LDS entries
  static_assert(BM % (16 * WR) == 0 && K % 32 == 0, "shape");
  static_assert(PF >= 1 && PF <= S && S % PF == 0, "the load ring must tile a work unit");
};

// LDS entry of the operand pair q (k = 8 g + 2 q, +1) of row block rb
// (within the block's BM rows) and step kb, for lane 0
template <class C>
__device__ __forceinline__ int frag(int rb, int kb, int q) {
  return ((rb * C::KB + kb) * 4 + q) * 64;
}

// rows row0 .. row0 + BM - 1 of E (row-major, K columns) into LDS
template <class C>
__device__ __forceinline__ void load_e(dv2* __restrict__ els, const double* __restrict__ E, int row0) {
#pragma unroll 4
  for (int c = threadIdx.x; c < C::PAIRS; c += C::NT) {
    const int lane = c & 63;
    int f = c >> 6;
    const int q = f & 3;
    f >>= 2;
    const int kb = f % C::KB, rb = f / C::KB;
    const int row = row0 + rb * 16 + (lane & 15);
    const int k = kb * 32 + 8 * (lane >> 4) + 2 * q;
    els[c] = *(const dv2*)(E + (long long)row * C::K + k);
  }
}

struct Ring8 {
  double v[8];
};

__device__ __forceinline__ void ld8(const double* __restrict__ p, Ring8& r) {
#pragma unroll
  for (int i = 0; i < 4; ++i) {
    const dv2 x = *(const dv2*)(p + 2 * i);
    r.v[2 * i] = x.x;
    r.v[2 * i + 1] = x.y;
  }
}

// a.L as a value the compiler cannot hoist products of out of the unit loop
__device__ __forceinline__ long long opaque_len(int L) {
  asm volatile("" : "+s"(L));
  return (long long)L;
}

// Work of one block: its row part, and its range [u0, u1) of units
// u = (b = u / CT, column tile u % CT).
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
  const int groups = gridDim.x / H;  // grid is a multiple of kXcd * H
  const int P = q * kXcd + x;
  w.CT = (L + C::COLS - 1) / C::COLS;
  const long long U = (long long)nfac * w.CT;
  w.u0 = U * P / groups;
  w.u1 = U * (P + 1) / groups;
  return w;
}

// load step t (0 <= t < S) of unit u into a ring slot
template <class C>
__device__ __forceinline__ void load_step(const double* __restrict__ X, long long xs, int L, const Work& w,
                                          long long u, int t, bool per_vector, Ring8 (&slot)[C::TN]) {
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int wc = wave % C::WC;
  const int v = t / C::KB, kb = t % C::KB;
  const int b = (int)(u / w.CT), ct = (int)(u % w.CT);
  const double* Xb = X + (per_vector ? (long long)v : (long long)b) * xs;
  const int k = kb * 32 + 8 * (lane >> 4);
#pragma unroll
  for (int c = 0; c < C::TN; ++c) {
    int j = ct * C::COLS + (wc * C::TN + c) * 16 + (lane & 15);
    j = j < L ? j : L - 1;
    ld8(Xb + (long long)j * C::K + k, slot[c]);
  }
}

// acc[rb][c] += A(rb, kb) B(c): the eight MFMAs of one 32-deep step per
// (row block, column block), ordered so that RB * TN independent
// accumulators separate two products into the same one.  The A pairs of the
// next pair index are read while this one's products run.
template <class C>
__device__ __forceinline__ void mma_step(const dv2* __restrict__ els, int kb, const Ring8 (&b)[C::TN],
                                         dacc (&acc)[C::RB][C::TN]) {
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int rb0 = (wave / C::WC) * C::RB;
  dv2 a[C::RB];
#pragma unroll
  for (int rb = 0; rb < C::RB; ++rb) a[rb] = els[frag<C>(rb0 + rb, kb, 0) + lane];
#pragma unroll
  for (int q = 0; q < 4; ++q) {
    dv2 n[C::RB];
    if (q + 1 < 4) {
#pragma unroll
      for (int rb = 0; rb < C::RB; ++rb) n[rb] = els[frag<C>(rb0 + rb, kb, q + 1) + lane];
    }
#pragma unroll
    for (int s = 0; s < 2; ++s)
#pragma unroll
      for (int rb = 0; rb < C::RB; ++rb)
#pragma unroll
        for (int c = 0; c < C::TN; ++c)
          acc[rb][c] = __builtin_amdgcn_mfma_f64_16x16x4f64(s ? a[rb].y : a[rb].x, b[c].v[2 * q + s], acc[rb][c], 0,
                                                            0, 0);
    __builtin_amdgcn_sched_barrier(0);
    if (q + 1 < 4) {
#pragma unroll
      for (int rb = 0; rb < C::RB; ++rb) a[rb] = n[rb];
    }
  }
}

// The shared driver: E reloads, the load ring across units, the MFMA steps;
// epi(u, w, acc) runs once per unit with the NV accumulator sets.
template <class C, class Epi>
__device__ __forceinline__ void run_units(const TtmArgs& a, bool per_vector, int nfac, dv2* __restrict__ els,
                                          Epi&& epi) {
  const Work w = block_work<C>(a.M, a.L, nfac);
  if (w.u0 >= w.u1) return;
  const double* X = (const double*)a.X;
  Ring8 ring[C::PF][C::TN];
#pragma unroll
  for (int t = 0; t < C::PF; ++t) load_step<C>(X, a.xs, a.L, w, w.u0, t, per_vector, ring[t]);
  int loaded = -1;
  for (long long u = w.u0; u < w.u1; ++u) {
    const int b = (int)(u / w.CT);
    const int fac = a.es == 0 ? 0 : b;
    if (fac != loaded) {
      __syncthreads();  // every wave is done with the previous factor
      load_e<C>(els, a.E + (long long)fac * a.es, w.h * C::BM);
      __syncthreads();
      loaded = fac;
    }
    dacc acc[C::NV][C::RB][C::TN];
#pragma unroll
    for (int v = 0; v < C::NV; ++v)
#pragma unroll
      for (int rb = 0; rb < C::RB; ++rb)
#pragma unroll
        for (int c = 0; c < C::TN; ++c) acc[v][rb][c] = (dacc){0.0, 0.0, 0.0, 0.0};
#pragma unroll
    for (int t = 0; t < C::S; ++t) {
      // the factor's pairs are the same for every vector of a unit: keep the
      // compiler from holding them all in registers across vectors
      asm volatile("" ::: "memory");
      const int slot = t % C::PF;
      Ring8 cur[C::TN];
#pragma unroll
      for (int c = 0; c < C::TN; ++c) cur[c] = ring[slot][c];
      const int tn = t + C::PF;
      if (tn < C::S)
        load_step<C>(X, a.xs, a.L, w, u, tn, per_vector, ring[slot]);
      else if (u + 1 < w.u1)
        load_step<C>(X, a.xs, a.L, w, u + 1, tn - C::S, per_vector, ring[slot]);
      mma_step<C>(els, t % C::KB, cur, acc[t / C::KB]);
    }
    epi(u, w, acc);
  }
}

// output row and column of accumulator element e of (row block rb, column
// block c) of this lane (D layout of the 16 x 16 x 4 FP64 MFMA: lane l,
// element e holds D[l / 16 + 4 e][l % 16])
template <class C>
__device__ __forceinline__ int out_row(const Work& w, int rb, int e) {
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  return w.h * C::BM + ((wave / C::WC) * C::RB + rb) * 16 + (lane >> 4) + 4 * e;
}
template <class C>
__device__ __forceinline__ int out_col(int ct, int c) {
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  return ct * C::COLS + ((wave % C::WC) * C::TN + c) * 16 + (lane & 15);
}

template <class C>
__global__ __launch_bounds__(C::NT) void ttm_f64r_store_kernel(TtmArgs a) {
  __shared__ dv2 els[C::PAIRS];
  if (a.stop && *a.stop) return;
  run_units<C>(a, false, a.nbatch, els, [&](long long u, const Work& w, dacc (&acc)[C::NV][C::RB][C::TN]) {
    const int b = (int)(u / w.CT), ct = (int)(u % w.CT);
    double* O = (double*)a.O + (long long)b * a.os;
    const long long L = opaque_len(a.L);
#pragma unroll
    for (int c = 0; c < C::TN; ++c) {
      const int col = out_col<C>(ct, c);
      if (col >= a.L) continue;
#pragma unroll
      for (int rb = 0; rb < C::RB; ++rb)
#pragma unroll
        for (int e = 0; e < 4; ++e) O[out_row<C>(w, rb, e) * L + col] = acc[0][rb][c][e];
    }
  });
}

// Squaring step (eq. squaring), NV orders per block: batch i is order
// o = i + 1 + order0 and O_i = 2^{-o} (E X_i + sum_{j=1}^{o} Y_j / (o-j)!),
// added to O_i when yacc is set; the NY = order0 + NV iterates Y_j are read
// once per element.
template <class C, int NY>
__global__ __launch_bounds__(C::NT) void ttm_f64r_square_kernel(TtmArgs a) {
  __shared__ dv2 els[C::PAIRS];
  if (a.stop && *a.stop) return;
  run_units<C>(a, true, 1, els, [&](long long u, const Work& w, dacc (&acc)[C::NV][C::RB][C::TN]) {
    const int ct = (int)(u % w.CT);
    const long long L = opaque_len(a.L);
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
            double s = acc[i][rb][c][e];
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

// Node sum fused into the last mode product (Algorithm 1): for every unit
// the block runs over the nbatch nodes b in turn, reloading factor b into
// LDS at each node (the load ring keeps streaming X across the reload), and
// keeps the NP running sums Y_q += 2^cexp coef[q][b] E_b X_b in registers.
template <class C, int NP>
__global__ __launch_bounds__(C::NT) void ttm_f64r_accum_kernel(TtmArgs a) {
  __shared__ dv2 els[C::PAIRS];
  if (a.stop && *a.stop) return;
  static_assert(C::NV == 1 && C::KB % C::PF == 0, "one node per step group; the ring tiles a node");
  const Work w = block_work<C>(a.M, a.L, 1);
  if (w.u0 >= w.u1) return;
  const double* X = (const double*)a.X;
  const int S = a.nbatch * C::KB;  // steps per unit
  Ring8 ring[C::PF][C::TN];
#pragma unroll
  for (int t = 0; t < C::PF; ++t) load_step<C>(X, a.xs, a.L, w, w.u0, t, true, ring[t]);
  for (long long u = w.u0; u < w.u1; ++u) {
    dacc y[NP][C::RB][C::TN];
#pragma unroll
    for (int q = 0; q < NP; ++q)
#pragma unroll
      for (int rb = 0; rb < C::RB; ++rb)
#pragma unroll
        for (int c = 0; c < C::TN; ++c) y[q][rb][c] = (dacc){0.0, 0.0, 0.0, 0.0};
    for (int b = 0; b < a.nbatch; ++b) {
      __syncthreads();  // every wave is done with the previous node's factor
      load_e<C>(els, a.E + (long long)b * a.es, w.h * C::BM);
      __syncthreads();
      dacc acc[C::RB][C::TN];
#pragma unroll
      for (int rb = 0; rb < C::RB; ++rb)
#pragma unroll
        for (int c = 0; c < C::TN; ++c) acc[rb][c] = (dacc){0.0, 0.0, 0.0, 0.0};
#pragma unroll
      for (int kb = 0; kb < C::KB; ++kb) {
        asm volatile("" ::: "memory");
        const int slot = kb % C::PF;  // = (b KB + kb) % PF
        Ring8 cur[C::TN];
#pragma unroll
        for (int c = 0; c < C::TN; ++c) cur[c] = ring[slot][c];
        const int tn = b * C::KB + kb + C::PF;
        if (tn < S)
          load_step<C>(X, a.xs, a.L, w, u, tn, true, ring[slot]);
        else if (u + 1 < w.u1)
          load_step<C>(X, a.xs, a.L, w, u + 1, tn - S, true, ring[slot]);
        mma_step<C>(els, kb, cur, acc);
      }
#pragma unroll
      for (int q = 0; q < NP; ++q) {
        const double wq = ldexp(a.coef[q * a.ldcoef + b], a.cexp);
#pragma unroll
        for (int rb = 0; rb < C::RB; ++rb)
#pragma unroll
          for (int c = 0; c < C::TN; ++c) y[q][rb][c] += wq * acc[rb][c];
      }
    }
    const int ct = (int)(u % w.CT);
    const long long L = opaque_len(a.L);
#pragma unroll
    for (int c = 0; c < C::TN; ++c) {
      const int col = out_col<C>(ct, c);
      if (col >= a.L) continue;
#pragma unroll
      for (int q = 0; q < NP; ++q) {
        double* Y = a.Y + q * a.ys;
#pragma unroll
        for (int rb = 0; rb < C::RB; ++rb)
#pragma unroll
          for (int e = 0; e < 4; ++e) {
            const long long idx = out_row<C>(w, rb, e) * L + col;
            Y[idx] = a.yacc ? Y[idx] + y[q][rb][c][e] : y[q][rb][c][e];
          }
      }
    }
  }
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

// Persistent grid: co-resident blocks, a multiple of kXcd * (row parts),
// at most one block per unit group.
template <class C, class F>
int grid_of(F kernel, int M, long long units) {
  static int per_cu = 0;
  if (!per_cu) {
    int b = 0;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&b, kernel, C::NT, 0) != hipSuccess || b < 1) b = 1;
    per_cu = b;
  }
  const int H = M / C::BM;
  long long g = (long long)cu_count() * per_cu;
  g = std::min<long long>(g, units * H);
  g = (g / (kXcd * H)) * (kXcd * H);
  return (int)(g < kXcd * H ? kXcd * H : g);
}

// shapes per n: (BM, WR, WC, TN).  n = 128: all rows per block, four waves
// of 16 columns each (64-column units: a single vector has one per CU);
// n = 256: a quarter of the rows; n = 64: all rows, four waves.
template <int K>
struct Shape;
template <>
struct Shape<64> {
  static constexpr int BM = 64, WR = 1, WC = 4, TN = 1;
};
template <>
struct Shape<128> {
  static constexpr int BM = 128, WR = 1, WC = 4, TN = 1;
};
template <>
struct Shape<256> {
  static constexpr int BM = 64, WR = 1, WC = 4, TN = 1;
};

// WR row groups (cfg 2: two, eight waves with half the row blocks each)
template <int K, int WR>
using StoreC = FC<Shape<K>::BM, K, WR, Shape<K>::WC, Shape<K>::TN, (K / 32 >= 4 ? 4 : K / 32), 1>;

template <class C>
int store_go(const TtmArgs& a, hipStream_t st) {
  auto k = ttm_f64r_store_kernel<C>;
  const long long units = (long long)a.nbatch * ((a.L + C::COLS - 1) / C::COLS);
  const int g = grid_of<C>(k, a.M, units);
  PHIQ_LAUNCH_F(k, dim3(g), dim3(C::NT), 0, st, a);
  return hipGetLastError();
}

template <int K>
int store_shape(const TtmArgs& a, hipStream_t st, int cfg) {
  // cfg 3: eight waves side by side (one row group, 128-column units);
  // cfg 4: sixteen (256-column units, two steps of loads in flight)
  using Wide = FC<Shape<K>::BM, K, 1, 8, Shape<K>::TN, (K / 32 >= 4 ? 4 : K / 32), 1>;
  using Wider = FC<Shape<K>::BM, K, 1, 16, Shape<K>::TN, (K / 32 >= 2 ? 2 : 1), 1>;
  // cfg 5: 64 rows per block (two row parts at n = 128, 64 KB of LDS: two
  // blocks per CU), eight waves side by side
  using Half = FC<64, K, 1, 8, 1, (K / 32 >= 4 ? 4 : K / 32), 1>;
  // cfg 6: 64 rows per block, sixteen waves side by side
  using HalfWide = FC<64, K, 1, 16, 1, (K / 32 >= 2 ? 2 : 1), 1>;
  if (cfg == 3) return store_go<Wide>(a, st);
  if (cfg == 4) return store_go<Wider>(a, st);
  if (cfg == 5) return store_go<Half>(a, st);
  if (cfg == 6) return store_go<HalfWide>(a, st);
  return cfg == 2 ? store_go<StoreC<K, 2>>(a, st) : store_go<StoreC<K, 1>>(a, st);
}

template <class C, int NY>
int square_go(const TtmArgs& a, hipStream_t st) {
  auto k = ttm_f64r_square_kernel<C, NY>;
  const long long units = (a.L + C::COLS - 1) / C::COLS;
  const int g = grid_of<C>(k, a.M, units);
  PHIQ_LAUNCH_F(k, dim3(g), dim3(C::NT), 0, st, a);
  return hipGetLastError();
}

// NV orders, NY = order0 + NV iterates (NY <= 4)
// (WR = 2: eight waves in two row groups, two waves per SIMD, so one wave's
// epilogue can run beside another's products; WC = 8: eight waves side by
// side)
template <int K, int NV, int WR, int WC = 4, int BM = Shape<K>::BM>
int square_nv(const TtmArgs& a, hipStream_t st) {
  constexpr int S = NV * (K / 32);
  using C = FC<BM, K, WR, WC, Shape<K>::TN, (S % 4 == 0 ? 4 : (S % 2 == 0 ? 2 : 1)), NV>;
  switch (a.order0 + NV) {
    case 1: return square_go<C, (NV <= 1 ? 1 : NV)>(a, st);
    case 2: return square_go<C, (NV <= 2 ? 2 : NV)>(a, st);
    case 3: return square_go<C, (NV <= 3 ? 3 : NV)>(a, st);
    default: return square_go<C, 4>(a, st);
  }
}

template <int K, int WR, int WC = 4, int BM = Shape<K>::BM>
int square_shape(const TtmArgs& a, hipStream_t st) {
  switch (a.nbatch) {
    case 1: return square_nv<K, 1, WR, WC, BM>(a, st);
    case 2: return square_nv<K, 2, WR, WC, BM>(a, st);
    case 3: return square_nv<K, 3, WR, WC, BM>(a, st);
    default: return square_nv<K, 4, WR, WC, BM>(a, st);
  }
}

// shapes the resident kernels take: FP64 in and out, rotated layout, M = K
// = n in {64, 128, 256}, 16-byte aligned operands, one batch stride per
// factor, no two-index batches
bool f64r_shape(const TtmArgs& a) {
  if (a.nn || a.x_f32 || a.o_f32 || a.M != a.K || !(a.K == 64 || a.K == 128 || a.K == 256)) return false;
  if (a.emod > 0 || a.xdiv > 0 || a.nouter > 1 || a.seg.n > 0 || a.L < 1 || a.nbatch < 1) return false;
  if (((uintptr_t)a.E | (uintptr_t)a.X) % 16 != 0) return false;
  if (a.es % 2 != 0 || a.xs % 2 != 0) return false;
  return true;
}

template <int K, int NP>
int accum_go(const TtmArgs& a, hipStream_t st) {
  using C = FC<Shape<K>::BM, K, 1, 8, Shape<K>::TN, (K / 32 >= 2 ? 2 : 1), 1>;
  auto k = ttm_f64r_accum_kernel<C, NP>;
  const long long units = (a.L + C::COLS - 1) / C::COLS;
  const int g = grid_of<C>(k, a.M, units);
  PHIQ_LAUNCH_F(k, dim3(g), dim3(C::NT), 0, st, a);
  return hipGetLastError();
}

template <int K>
int accum_shape(const TtmArgs& a, hipStream_t st) {
  switch (a.np) {
    case 1: return accum_go<K, 1>(a, st);
    case 2: return accum_go<K, 2>(a, st);
    case 3: return accum_go<K, 3>(a, st);
    default: return accum_go<K, 4>(a, st);
  }
}

}  // namespace

int f64r_num_configs() { return 7; }
int f64r_accum_num_configs() { return 2; }

// Node sum: cfg 1 = the resident kernel (eight waves side by side), 0 or -1
// (default) = decline.  At n = 256 (eight nodes, three running sums, one
// factor reload per node and unit) it measured 1.38-1.39 ms per 3D
// phi-action against 1.35-1.36 ms for the tile kernel; at n = 128 its
// running sums spill.
int launch_ttm_accum_f64r(const TtmArgs& a, void* stream, int cfg) {
  if (cfg <= 0 || !f64r_shape(a) || a.np < 1 || a.np > 4) return hipErrorNotSupported;
  hipStream_t st = (hipStream_t)stream;
  if (a.K == 256) return accum_shape<256>(a, st);
  if (a.K == 128) return accum_shape<128>(a, st);
  return accum_shape<64>(a, st);
}

// cfg: 0 = decline (the caller runs the tile kernels), 1 = four waves with
// all row blocks each, 2 = eight waves in two row groups (both 64-column
// units), 3 = eight waves in one row group (128-column units), 4 = sixteen
// waves in one row group (256-column units), 5 = eight waves on 64-row
// blocks, 6 = sixteen waves on 64-row blocks, -1 = default: cfg 4 at n = 256
// with at least one unit per CU, cfg 6 at n = 128 for batches of eight or
// more, else decline.  Measured on gfx950 against
// the tile kernels (per launch): n = 256, one vector 143-153 us (cfg 4),
// 148-166 (cfg 3), 156-165 (cfg 2) against 162-169; three vectors 396-404
// (cfg 4), 408-412 (cfg 3), 436-462 (cfg 2) against 447-472;
// n = 128, one vector 21 us against 17 (the fixed cost of filling 128 KB of
// LDS and the load ring is not repaid by 7 us of matrix work), eight vectors
// 95 against 91; n = 64 slower still.  Returns hipErrorNotSupported for
// launches the resident kernels do not take.
int launch_ttm_store_f64r(const TtmArgs& a, void* stream, int cfg) {
  if (cfg == 0 || !f64r_shape(a)) return hipErrorNotSupported;
  const int H = a.K == 256 ? 4 : 1;
  const long long units = (long long)a.nbatch * ((a.L + 63) / 64) * H;
  if (cfg < 0) {
    // n = 256: sixteen waves; n = 128 with eight or more vectors (a node
    // batch): 64 rows per block, sixteen waves, 100-107 us against 114-117
    // us for ten vectors (eight waves: 106-116 us; one to three vectors
    // stay faster on the tile kernel)
    if (a.K == 256 && units >= cu_count())
      cfg = 4;
    else if (a.K == 128 && a.nbatch >= 8)
      cfg = 6;
    else
      return hipErrorNotSupported;
  }
  hipStream_t st = (hipStream_t)stream;
  if (a.K == 256) return store_shape<256>(a, st, cfg);
  if (a.K == 128) return store_shape<128>(a, st, cfg);
  return store_shape<64>(a, st, cfg);
}

// Squaring: cfg 1 = the resident kernel (four waves), 2 = eight waves in two
// row groups, 3 = eight waves in one row group, 0 = decline, -1 = default:
// cfg 3 at n = 256 with at least one unit per CU, else decline.  Per 3D
// phi-action (seven three-order steps at n = 256, five at n = 128): n = 256
// 3.26-3.29 ms (cfg 3), 3.40-3.46 (cfg 2) and 4.04 (cfg 1) against 3.73 ms
// with the tile kernel; n = 128 0.23 / 0.24 (cfg 2 / 1) against 0.21, and
// the one-group shapes spill registers there (all rows per wave).
int launch_ttm_square_f64r(const TtmArgs& a, void* stream, int cfg) {
  if (cfg == 0 || !f64r_shape(a) || a.nbatch > 4 || a.es != 0 || a.order0 < 0 || a.order0 + a.nbatch > 4 ||
      a.yps % 2 != 0 || (a.nbatch > 1 && a.os % 2 != 0))
    return hipErrorNotSupported;
  if (cfg < 0) {
    const long long units = (long long)((a.L + 63) / 64) * (a.K == 256 ? 4 : 1);
    if (a.K != 256 || units < cu_count()) return hipErrorNotSupported;
    cfg = 3;
  }
  hipStream_t st = (hipStream_t)stream;
  if (cfg == 4) {  // 64 rows per block, eight waves side by side
    if (a.K == 256) return square_shape<256, 1, 8, 64>(a, st);
    if (a.K == 128) return square_shape<128, 1, 8, 64>(a, st);
    return square_shape<64, 1, 8, 64>(a, st);
  }
  if (cfg == 3) {
    if (a.K == 256) return square_shape<256, 1, 8>(a, st);
    if (a.K == 128) return square_shape<128, 1, 8>(a, st);
    return square_shape<64, 1, 8>(a, st);
  }
  if (cfg == 2) {
    if (a.K == 256) return square_shape<256, 2>(a, st);
    if (a.K == 128) return square_shape<128, 2>(a, st);
    return square_shape<64, 2>(a, st);
  }
  if (a.K == 256) return square_shape<256, 1>(a, st);
  if (a.K == 128) return square_shape<128, 1>(a, st);
  return square_shape<64, 1>(a, st);
}

}  // namespace phiq
