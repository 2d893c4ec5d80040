// Two mode products per slab (gfx950, v_mfma_f64_16x16x4_f64), for tensors
// whose two fastest axes both have 128 points.
//
// A tensor x[i0][i1][i2] is n0 slabs of 128 x 128.  On slab i0 the products
// along axes 2 and 1 (eq. Expkron: the factors act on their own axis only)
// are two 128-deep contractions:
//   Y1[i1][j2] = sum_k  X[i1][k]  E2[j2][k]        (axis 2)
//   Y2[j1][j2] = sum_k  E1[j1][k] Y1[k][j2]        (axis 1)
// and Y2 is written back in the same layout, so the product along axis 0
// then reads the tensor in its natural layout.  One pass over HBM does the
// work of two single-axis passes.
//
// Work split.  A task is one half of a slab (64 of the 128 output columns
// j2); a block of four waves takes one task at a time, wave w the 16
// columns 64 h + 16 w.. of its half.  Each wave computes the full 128 rows
// of Y1 for its columns into eight accumulator tiles.  The MFMA output
// layout (lane l, element e holds row l/16 + 4e, column l%16 of a 16 x 16
// tile) is exactly the B-operand layout of a 4-deep k-step (lane l holds
// row l/16, column l%16), so element e of Y1's tile r is the B operand for
// k = 16 r + 4 e .. +3 of the second product: Y1 never leaves registers.
//
// Operands.  E1 (A operand of the second product) sits in LDS for the
// block's whole run of slabs of one batch entry, 128 KB in fragment order
// (the 64 doubles a wave reads for one 16 x 4 fragment are contiguous).
// E2 (B operand of the first product) stays in registers: the wave's 16
// columns, all 128 k, 32 doubles per lane.  X is staged through LDS in
// 16-deep k chunks (16 KB, double-buffered), also in fragment order, with
// the lane index XOR-ed by 8 kq so that the chunk writes spread over the
// banks.  The next slab's first chunk is loaded during the current slab's
// second product.
//
// Scheduling.  The two blocks that take the halves of one slab are given
// block ids g and g + 8, which the hardware deals to the same XCD, so the
// second read of the slab is served by that XCD's L2.  Every block pair
// takes a contiguous run of slabs (slab s = batch entry s / n0, i0 = s % n0),
// so the factors change at most a few times per block.
#include <hip/hip_ext.h>
#include <hip/hip_runtime.h>

#include "phiq_internal.h"

#define PHIQ_SLAB_LAUNCH(K, G, B, SH, ST, ...)                                                            \
  do {                                                                                                    \
    if (g_launch_events[0])                                                                               \
      hipExtLaunchKernelGGL(K, G, B, SH, ST, (hipEvent_t)g_launch_events[0], (hipEvent_t)g_launch_events[1], \
                            0, __VA_ARGS__);                                                              \
    else                                                                                                  \
      hipLaunchKernelGGL(K, G, B, SH, ST, __VA_ARGS__);                                                   \
  } while (0)

namespace phiq {
namespace {

typedef double d4 __attribute__((ext_vector_type(4)));
typedef double d2 __attribute__((ext_vector_type(2)));

constexpr int S = kSlabN;   // points on each of the two fast axes
constexpr int CK = 16;      // k per staged X chunk
constexpr int NCH = S / CK; // chunks per slab
constexpr int NT = 256;     // four waves
constexpr int XPER = S * CK / 2 / NT;  // 16-byte X loads per thread per chunk (4)

// X chunk c of a slab (rows i1, k = 16 c ..): thread t loads pairs
// t + 256 u: row (t + 256 u) / 8, k pair (t + 256 u) % 8.
__device__ __forceinline__ void load_chunk(const double* __restrict__ xb, int c, d2 (&pf)[XPER]) {
#pragma unroll
  for (int u = 0; u < XPER; ++u) {
    const int pi = threadIdx.x + NT * u;
    const int r = pi >> 3, kp = pi & 7;
    pf[u] = *(const d2*)(xb + r * S + CK * c + 2 * kp);
  }
}

// Fragment (ia, kq) of a chunk holds X[16 ia + l%16][4 kq + l/16] at lane
// l ^ 8 kq of a 64-double block.
__device__ __forceinline__ void store_chunk(double* __restrict__ xs, const d2 (&pf)[XPER]) {
#pragma unroll
  for (int u = 0; u < XPER; ++u) {
    const int pi = threadIdx.x + NT * u;
    const int r = pi >> 3, kp = pi & 7;
    const int kq = kp >> 1;
    const int ll = (r & 15) + 32 * (kp & 1);  // logical lane of the pair's first element
    double* base = xs + ((r >> 4) * 4 + kq) * 64;
    base[ll ^ (8 * kq)] = pf[u].x;
    base[(ll + 16) ^ (8 * kq)] = pf[u].y;
  }
}

// The 32 A operands (8 row tiles x 4 k-steps) of one staged chunk.
__device__ __forceinline__ void read_chunk_ops(const double* __restrict__ xs, int lane, double (&op)[32]) {
#pragma unroll
  for (int kq = 0; kq < 4; ++kq)
#pragma unroll
    for (int ia = 0; ia < 8; ++ia) op[kq * 8 + ia] = xs[(ia * 4 + kq) * 64 + (lane ^ (8 * kq))];
}
// The 32 A operands of E1 for k-steps 4 kb .. 4 kb + 3 of the second product.
__device__ __forceinline__ void read_e1_ops(const double* __restrict__ e1s, int kb, int lane, double (&op)[32]) {
#pragma unroll
  for (int e = 0; e < 4; ++e)
#pragma unroll
    for (int ia = 0; ia < 8; ++ia) op[e * 8 + ia] = e1s[(ia * 32 + 4 * kb + e) * 64 + lane];
}

__global__ __launch_bounds__(NT, 1) void slab2_kernel(SlabArgs a) {
  __shared__ double e1s[S * S];       // E1 in A-fragment order: ((ia * 32 + kk) * 64 + lane)
  __shared__ double xs[2][S * CK];    // X chunks in A-fragment order
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  const int g = blockIdx.x;
  const int Q = gridDim.x / 2;                  // block pairs
  const int q = (g & 7) + 8 * ((g >> 3) >> 1);  // blocks g and g + 8 form pair q
  const int h = (g >> 3) & 1;
  const long long nslab = (long long)a.n0 * a.nbatch;
  const long long cnt = (nslab + Q - 1) / Q;
  const long long s0 = (long long)q * cnt;
  const long long s1 = s0 + cnt < nslab ? s0 + cnt : nslab;
  if (s0 >= s1) return;  // uniform per block
  const int col = 64 * h + 16 * w + (lane & 15);  // this lane's output column j2 (B operand / output)
  auto slab_x = [&](long long s) {
    const long long b = s / a.n0, i0 = s - b * a.n0;
    return a.X + b * a.xs + i0 * S * S;
  };

  const double* curE1 = nullptr;
  const double* curE2 = nullptr;
  double e2r[S / 4];  // E2[col][4 kk + lane/16], kk = 0..31
  // chunk j of the slab travels in pf[j & 1], two chunks ahead of its use
  d2 pf[2][XPER];
  load_chunk(slab_x(s0), 0, pf[0]);
  load_chunk(slab_x(s0), 1, pf[1]);
  for (long long s = s0; s < s1; ++s) {
    const long long b = s / a.n0, i0 = s - b * a.n0;
    const double* xb = slab_x(s);
    const double* E1 = a.E1 + b * a.es1;
    const double* E2 = a.E2 + b * a.es2;
    __syncthreads();  // the previous slab's readers of e1s and xs are done
    if (E2 != curE2) {
#pragma unroll
      for (int kk = 0; kk < S / 4; ++kk) e2r[kk] = E2[col * S + 4 * kk + (lane >> 4)];
      curE2 = E2;
    }
    if (E1 != curE1) {
      // pair (row 16 ia + j % 16, columns 4 kk + 2 (j / 16) ..+1) of fragment
      // f = (ia, kk), j < 32; sixteen loads in flight, then their writes
      constexpr int EU = S * S / 2 / NT, EB = 16;
#pragma unroll
      for (int u0 = 0; u0 < EU; u0 += EB) {
        d2 v[EB];
#pragma unroll
        for (int u = 0; u < EB; ++u) {
          const int pi = threadIdx.x + NT * (u0 + u);
          const int f = pi >> 5, jj = pi & 31;
          v[u] = *(const d2*)(E1 + (16 * (f >> 5) + (jj & 15)) * S + 4 * (f & 31) + 2 * (jj >> 4));
        }
        __builtin_amdgcn_sched_barrier(0);
#pragma unroll
        for (int u = 0; u < EB; ++u) {
          const int pi = threadIdx.x + NT * (u0 + u);
          const int f = pi >> 5, jj = pi & 31;
          e1s[f * 64 + (jj & 15) + 32 * (jj >> 4)] = v[u].x;
          e1s[f * 64 + (jj & 15) + 32 * (jj >> 4) + 16] = v[u].y;
        }
      }
      curE1 = E1;
    }
    store_chunk(xs[0], pf[0]);
    load_chunk(xb, 2, pf[0]);
    __syncthreads();

    // Y1 = X E2^T for this wave's 16 columns, all 128 rows.  Chunk c sits in
    // xs[c & 1]; its A operands are read one chunk ahead of its MFMAs.
    d4 y1[8];
#pragma unroll
    for (int i = 0; i < 8; ++i) y1[i] = (d4){0.0, 0.0, 0.0, 0.0};
    double op[2][32];
    read_chunk_ops(xs[0], lane, op[0]);
    store_chunk(xs[1], pf[1]);  // nobody reads xs[1] before the next barrier
    load_chunk(xb, 3, pf[1]);
#pragma unroll
    for (int c = 0; c < NCH; ++c) {
      // chunk c + 1 is visible; every wave's reads of chunk c (xs[c & 1]) are done
      __syncthreads();
      if (c + 1 < NCH) read_chunk_ops(xs[(c + 1) & 1], lane, op[(c + 1) & 1]);
      __builtin_amdgcn_sched_barrier(0);
#pragma unroll
      for (int kq = 0; kq < 4; ++kq)
#pragma unroll
        for (int ia = 0; ia < 8; ++ia)
          y1[ia] = __builtin_amdgcn_mfma_f64_16x16x4f64(op[c & 1][kq * 8 + ia], e2r[4 * c + kq], y1[ia], 0, 0, 0);
      __builtin_amdgcn_sched_barrier(0);
      // after the MFMAs are issued, so that a late global load does not hold them up
      if (c + 2 < NCH) {
        store_chunk(xs[c & 1], pf[c & 1]);  // chunk c + 2
        if (c + 4 < NCH)
          load_chunk(xb, c + 4, pf[c & 1]);
        else if (s + 1 < s1)  // the next slab's chunk c + 4 - NCH
          load_chunk(slab_x(s + 1), c + 4 - NCH, pf[c & 1]);
      }
    }

    // Y2 = E1 Y1: element e of Y1 tile kb is the B operand of k-step 4 kb + e;
    // the E1 operands of k-block kb + 1 are read during k-block kb
    d4 y2[8];
#pragma unroll
    for (int i = 0; i < 8; ++i) y2[i] = (d4){0.0, 0.0, 0.0, 0.0};
    read_e1_ops(e1s, 0, lane, op[0]);
#pragma unroll
    for (int kb = 0; kb < 8; ++kb) {
      if (kb + 1 < 8) read_e1_ops(e1s, kb + 1, lane, op[(kb + 1) & 1]);
      __builtin_amdgcn_sched_barrier(0);
#pragma unroll
      for (int e = 0; e < 4; ++e)
#pragma unroll
        for (int ia = 0; ia < 8; ++ia)
          y2[ia] = __builtin_amdgcn_mfma_f64_16x16x4f64(op[kb & 1][e * 8 + ia], y1[kb][e], y2[ia], 0, 0, 0);
      __builtin_amdgcn_sched_barrier(0);
    }

    double* ob = a.O + b * a.os + i0 * S * S + col;
#pragma unroll
    for (int ia = 0; ia < 8; ++ia)
#pragma unroll
      for (int e = 0; e < 4; ++e) ob[(16 * ia + (lane >> 4) + 4 * e) * S] = y2[ia][e];
  }
}

}  // namespace

bool slab2_supported(const SlabArgs& a) {
  const uintptr_t al = (uintptr_t)a.X | (uintptr_t)a.E1 | (uintptr_t)a.E2;
  return a.n0 >= 1 && a.nbatch >= 1 && al % 16 == 0 && a.xs % 2 == 0 && a.es1 % 2 == 0 && a.es2 % 2 == 0;
}

int launch_slab2(const SlabArgs& a, void* stream) {
  if (!slab2_supported(a)) return hipErrorInvalidValue;
  const long long nslab = (long long)a.n0 * a.nbatch;
  // one block per CU (the block holds 160 KB of LDS); pairs of blocks in
  // multiples of 8 so that both halves of a slab land on one XCD
  const long long pairs = nslab < 128 ? nslab : 128;
  const long long blocks = (2 * pairs + 15) / 16 * 16;
  PHIQ_SLAB_LAUNCH(slab2_kernel, dim3((unsigned)blocks), dim3(NT), 0, (hipStream_t)stream, a);
  return hipGetLastError();
}

}  // namespace phiq
