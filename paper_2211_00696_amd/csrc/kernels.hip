// HIP kernels for gfx950 (CDNA4): FP64 MFMA mode products with fused
// node-sum and squaring epilogues, small batched GEMMs and the truncated
// Taylor series used for the 1D exponentials.
//
// MFMA building block: v_mfma_f64_16x16x4_f64 (one wave, 64 lanes).
//   A operand: lane l holds A[l % 16][l / 16]      (16 x 4)
//   B operand: lane l holds B[l / 16][l % 16]      (4 x 16)
//   D (4 doubles): lane l, element e holds D[l / 16 + 4 e][l % 16]
#include <hip/hip_ext.h>
#include <hip/hip_runtime.h>

#include "phiq_internal.h"
#include "tile_fp64.h"

namespace phiq {

thread_local void* g_launch_events[2] = {nullptr, nullptr};

// Launch, with the live-timing events attached when they are set.
#define PHIQ_LAUNCH(K, G, B, SH, ST, ...)                                                                 \
  do {                                                                                                    \
    if (g_launch_events[0])                                                                               \
      hipExtLaunchKernelGGL(K, G, B, SH, ST, (hipEvent_t)g_launch_events[0], (hipEvent_t)g_launch_events[1], \
                            0, __VA_ARGS__);                                                              \
    else                                                                                                  \
      hipLaunchKernelGGL(K, G, B, SH, ST, __VA_ARGS__);                                                   \
  } while (0)

// ---------------------------------------------------------------------------
// Mode products (rotated layout), three epilogues.
//
// Main loop: register prefetch two chunks ahead and a double-buffered LDS
// tile, one barrier per K-chunk.  Blocks are mapped to tiles XCD-aware: the
// hardware deals consecutive block ids round-robin to the 8 XCDs, so block b
// takes tile (b % 8) * ceil(T/8) + b / 8 and the M-tiles of one column block
// (which read the same X rows) share an XCD's L2.
// ---------------------------------------------------------------------------
constexpr int kXcds = 8;

// Tile of this block: returns false for the padding blocks of the last XCD.
// Tiles are numbered (M tile, batch, column block), M tile fastest.
template <class C>
__device__ __forceinline__ bool tile_of_block(int M, int L, int nb, int& m0, int& n0, int& b) {
  const long long T = ttm_tiles<C>(M, L, nb);
  const long long per = (T + kXcds - 1) / kXcds;
  const long long t = (long long)(blockIdx.x % kXcds) * per + blockIdx.x / kXcds;
  if (t >= T) return false;
  // M tile fastest, then batch, then column block: the blocks that share an
  // X tile (M tiles; batches when X is shared) or the y_j tiles read by the
  // squaring epilogue run back to back on one XCD
  const int mtiles = (M + C::BM - 1) / C::BM;
  m0 = (int)(t % mtiles) * C::BM;
  const long long r = t / mtiles;
  b = (int)(r % nb);
  n0 = (int)(r / nb) * C::BN;
  return true;
}

template <class C, bool VEC, bool NN = false>
__global__ __launch_bounds__(C::NT, C::MINW) void ttm_store_kernel(TtmArgs a) {
  __shared__ double smem[2 * (C::BM + C::BN) * C::LDK];
  if (a.stop && *a.stop) return;
  int m0, n0, b;
  if (!tile_of_block<C>(a.M, a.L, a.nbatch, m0, n0, b)) return;
  int be = a.emod > 0 ? b % a.emod : b;
  int bx = a.xdiv > 0 ? b / a.xdiv : b;
  const double* X = (const double*)a.X;
  if (a.seg.n > 0) {
    // constant indices only: the table stays in the argument segment
    int s0 = a.seg.sb[0], e0 = a.seg.se[0];
    const double* x0 = a.seg.sx[0];
#pragma unroll
    for (int s = 1; s < kSegMax; ++s)
      if (s < a.seg.n && b >= a.seg.sb[s]) {
        s0 = a.seg.sb[s];
        e0 = a.seg.se[s];
        x0 = a.seg.sx[s];
      }
    be = e0 + (b - s0);
    if (x0) {
      X = x0;
      bx = 0;
    }
  }
  d4 acc[C::TM][C::TN];
  zero_acc<C>(acc);
  tile_nt_db<C, VEC, NN>(a.E + be * a.es, X + bx * a.xs, a.M, a.K, a.L, m0, n0, smem, acc);
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
// nodes b and keeps the NP running sums in registers.
template <class C, int NP, bool VEC, bool NN = false>
__global__ __launch_bounds__(C::NT, C::MINW) void ttm_accum_kernel(TtmArgs a) {
  __shared__ double smem[2 * (C::BM + C::BN) * C::LDK];
  int m0, n0, r;
  if (!tile_of_block<C>(a.M, a.L, a.nouter > 1 ? a.nouter : 1, m0, n0, r)) return;
  const double* X = (const double*)a.X + r * a.xo;
  d4 y[NP][C::TM][C::TN];
#pragma unroll
  for (int q = 0; q < NP; ++q) zero_acc<C>(y[q]);
  for (int b = 0; b < a.nbatch; ++b) {
    d4 acc[C::TM][C::TN];
    zero_acc<C>(acc);
    tile_nt_db<C, VEC, NN>(a.E + (a.emod > 0 ? b % a.emod : b) * a.es, X + b * a.xs, a.M, a.K, a.L, m0, n0, smem,
                           acc);
#pragma unroll
    for (int q = 0; q < NP; ++q) {
      const double w = ldexp(a.coef[q * a.ldcoef + b], a.cexp);
#pragma unroll
      for (int i = 0; i < C::TM; ++i)
#pragma unroll
        for (int j = 0; j < C::TN; ++j) y[q][i][j] += w * acc[i][j];
    }
  }
#pragma unroll
  for (int q = 0; q < NP; ++q) {
    double* Y = a.Y + r * a.yo + q * a.ys;
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
            Y[idx] = a.yacc ? Y[idx] + y[q][i][j][e] : y[q][i][j][e];
          }
        }
      }
  }
}

// Modified squaring fused into the last mode product (eq. squaring):
// batch b is order i = b+1+order0, out = 2^{-i} (E y_i + sum_{j=1}^{i} y_j/(i-j)!),
// added to out when yacc is set.
template <class C, bool VEC, bool NN = false>
__global__ __launch_bounds__(C::NT, C::MINW) void ttm_square_kernel(TtmArgs a) {
  __shared__ double smem[2 * (C::BM + C::BN) * C::LDK];
  int m0, n0, bt;
  const int no = a.nouter > 1 ? a.nouter : 1;
  if (!tile_of_block<C>(a.M, a.L, a.nbatch * no, m0, n0, bt)) return;
  const int r = bt / a.nbatch, b = bt % a.nbatch;
  d4 acc[C::TM][C::TN];
  zero_acc<C>(acc);
  tile_nt_db<C, VEC, NN>(a.E + b * a.es, (const double*)a.X + r * a.xo + b * a.xs, a.M, a.K, a.L, m0, n0, smem,
                         acc);
  const int order = b + 1 + a.order0;
  const double scale = ldexp(1.0, -order);
  double* O = (double*)a.O + r * a.oo + b * a.os;
  const double* Yp = a.Yprev + r * a.ypo;
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
          for (int jj = 1; jj <= order; ++jj) s += Yp[(jj - 1) * a.yps + idx] * a.ifact[order - jj];
          O[idx] = a.yacc ? O[idx] + scale * s : scale * s;
        }
      }
    }
}

// All p orders of one modified-squaring step in one block (p <= 4): the
// block computes E y_i for i = 1..p in turn and reads every y_j tile once,
// keeping it in registers for the later orders.  Same factor E for all i.
template <class C, int NP, bool VEC, bool NN = false>
__global__ __launch_bounds__(C::NT, C::MINW) void ttm_square_all_kernel(TtmArgs a) {
  __shared__ double smem[2 * (C::BM + C::BN) * C::LDK];
  int m0, n0, r;
  if (!tile_of_block<C>(a.M, a.L, a.nouter > 1 ? a.nouter : 1, m0, n0, r)) return;
  const double* X = (const double*)a.X + r * a.xo;
  const double* Yp = a.Yprev + r * a.ypo;
  d4 ys[NP][C::TM][C::TN];
#pragma unroll
  for (int i = 0; i < NP; ++i) {
    // y_{i+1} tile: issued before the K loop so it arrives during it
#pragma unroll
    for (int ti = 0; ti < C::TM; ++ti)
#pragma unroll
      for (int tj = 0; tj < C::TN; ++tj) {
        const int col = n0 + acc_col<C>(tj);
#pragma unroll
        for (int e = 0; e < 4; ++e) {
          const int row = m0 + acc_row<C>(ti, e);
          const int rc = row < a.M ? row : a.M - 1, cc = col < a.L ? col : a.L - 1;
          ys[i][ti][tj][e] = Yp[i * a.yps + (long long)rc * a.L + cc];
        }
      }
    d4 acc[C::TM][C::TN];
    zero_acc<C>(acc);
    tile_nt_db<C, VEC, NN>(a.E, X + i * a.xs, a.M, a.K, a.L, m0, n0, smem, acc);
    const double scale = ldexp(1.0, -(i + 1));
    double* O = (double*)a.O + r * a.oo + i * a.os;
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
          for (int j = 0; j <= i; ++j) s += ys[j][ti][tj][e] * a.ifact[i - j];
          if (row < a.M && col < a.L) O[(long long)row * a.L + col] = scale * s;
        }
      }
  }
}

// ---------------------------------------------------------------------------
// Small batched GEMM C = A B (n x n), one job per blockIdx.z.
// ---------------------------------------------------------------------------
template <class C>
__global__ __launch_bounds__(C::NT) void gemm_jobs_kernel(const GemmJob* __restrict__ jobs, const int* __restrict__ stop) {
  __shared__ double As[C::BM * C::LDK];
  __shared__ double Bs[C::BN * C::LDK];
  if (stop && *stop) return;
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

// The same for n <= kPanelK: a block loads its whole 32-row panel of A and
// 32-column panel of B in one pass (every load in flight at once, one
// barrier), then four waves take a 16 x 16 quarter of the 32 x 32 output
// each.  The k order of the MFMA chain is the one above (which only adds
// zero products past n), so the two kernels agree up to the sign of exact
// zeros; this one pays one load latency per block instead of one per
// 16-deep chunk.
constexpr int kPanelK = 128;
__global__ __launch_bounds__(256) void gemm_panel_kernel(const GemmJob* __restrict__ jobs, const int* __restrict__ stop) {
  constexpr int BM = 32, BN = 32, LDK = kPanelK + 2, NT = 256, PER = BM * kPanelK / NT;
  __shared__ double As[BM * LDK];
  __shared__ double Bs[BN * LDK];
  if (stop && *stop) return;
  const GemmJob jb = jobs[blockIdx.z];
  const int n = jb.n;
  const int m0 = blockIdx.x * BM, n0 = blockIdx.y * BN;
  if (m0 >= n || n0 >= n) return;  // uniform per block
  double ra[PER], rb[PER];
#pragma unroll
  for (int i = 0; i < PER; ++i) {
    const int e = threadIdx.x + i * NT;
    const int r = m0 + e / kPanelK, k = e % kPanelK;  // A: k fastest
    ra[i] = (r < n && k < n) ? jb.A[(long long)r * n + k] : 0.0;
    const int kb = e / BN, c = n0 + e % BN;  // B: columns fastest
    rb[i] = (kb < n && c < n) ? jb.B[(long long)kb * n + c] : 0.0;
  }
#pragma unroll
  for (int i = 0; i < PER; ++i) {
    const int e = threadIdx.x + i * NT;
    As[(e / kPanelK) * LDK + e % kPanelK] = ra[i];
    Bs[(e % BN) * LDK + e / BN] = rb[i];
  }
  __syncthreads();
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int wm = wave >> 1, wn = wave & 1;
  const double* a = As + (16 * wm + (lane & 15)) * LDK + (lane >> 4);
  const double* b = Bs + (16 * wn + (lane & 15)) * LDK + (lane >> 4);
  d4 acc = {0.0, 0.0, 0.0, 0.0};
  const int ksteps = (n + 3) / 4;
  for (int k4 = 0; k4 < ksteps; ++k4) acc = __builtin_amdgcn_mfma_f64_16x16x4f64(a[4 * k4], b[4 * k4], acc, 0, 0, 0);
  const int col = n0 + 16 * wn + (lane & 15);
#pragma unroll
  for (int e = 0; e < 4; ++e) {
    const int row = m0 + 16 * wm + (lane >> 4) + 4 * e;
    if (row < n && col < n) jb.C[(long long)row * n + col] = acc[e];
  }
}

__global__ void scale_jobs_kernel(const ScaleJob* __restrict__ jobs, const int* __restrict__ stop) {
  if (stop && *stop) return;
  const ScaleJob jb = jobs[blockIdx.y];
  const long long nn = (long long)jb.n * jb.n;
  for (long long i = blockIdx.x * (long long)blockDim.x + threadIdx.x; i < nn; i += (long long)gridDim.x * blockDim.x)
    jb.dst[i] = jb.s * jb.src[i];
}

// dst[t] = I + sum_{k=1}^{K} c_t^k/k! Z^k by Horner's rule in c_t:
//   c (Z + c/2 (Z^2 + c/3 (Z^3 + ...))),
// with the K powers of one element held in registers for all targets.
__global__ __launch_bounds__(256) void taylor_jobs_kernel(const TaylorJob* __restrict__ jobs, const int* __restrict__ stop) {
  if (stop && *stop) return;
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
                                   long long N, double* __restrict__ partial, const int* __restrict__ stop) {
  __shared__ double sd[256], sy[256];
  if (stop && *stop) return;
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
// NP > 0: that many outputs, kept in registers; NP = 0: np outputs (any).
template <int NP>
__global__ void node_sum_kernel(NodeSegs segs, long long N, const double* __restrict__ coef, int ldcoef, int np,
                                double* __restrict__ Y, const int* __restrict__ stop) {
  constexpr int A = NP > 0 ? NP : PHIQ_MAX_P;
  if (stop && *stop) return;
  const int n = NP > 0 ? NP : np;
  for (long long i = blockIdx.x * (long long)blockDim.x + threadIdx.x; i < N; i += (long long)gridDim.x * blockDim.x) {
    double acc[A];
#pragma unroll
    for (int j = 0; j < A; ++j) acc[j] = 0.0;
    int b = 0;
    for (int sg = 0; sg < segs.nseg; ++sg) {
      const double* V = segs.V[sg];
      for (int c = 0; c < segs.count[sg]; ++c, ++b) {
        const double x = V[(long long)c * N + i];
#pragma unroll
        for (int j = 0; j < A; ++j)
          if (j < n) acc[j] += coef[j * ldcoef + b] * x;
      }
    }
#pragma unroll
    for (int j = 0; j < A; ++j)
      if (j < n) Y[j * N + i] = acc[j];
  }
}

// One block: the relative change of Algorithm 2 from the absdiff partial
// maxima, and whether it meets tol (or an earlier level already did).
__global__ __launch_bounds__(256) void cc_decide_kernel(const double* __restrict__ partial, int nblk, int np,
                                                        double tol, const int* __restrict__ prev,
                                                        CcCtl* __restrict__ out) {
  __shared__ double sn[256], sd[256];
  if (prev && *prev) {
    if (threadIdx.x == 0) {
      out->err = -1.0;
      out->stop = 1;
    }
    return;
  }
  double err = 0.0;
  for (int j = 0; j < np; ++j) {
    double num = 0.0, den = 0.0;
    for (int b = threadIdx.x; b < nblk; b += blockDim.x) {
      num = fmax(num, partial[((long long)b * np + j) * 2 + 0]);
      den = fmax(den, partial[((long long)b * np + j) * 2 + 1]);
    }
    sn[threadIdx.x] = num;
    sd[threadIdx.x] = den;
    __syncthreads();
    for (int s = blockDim.x / 2; s > 0; s >>= 1) {
      if ((int)threadIdx.x < s) {
        sn[threadIdx.x] = fmax(sn[threadIdx.x], sn[threadIdx.x + s]);
        sd[threadIdx.x] = fmax(sd[threadIdx.x], sd[threadIdx.x + s]);
      }
      __syncthreads();
    }
    err = fmax(err, sd[0] > 0.0 ? sn[0] / sd[0] : sn[0]);
    __syncthreads();
  }
  if (threadIdx.x == 0) {
    out->err = err;
    out->stop = err <= tol ? 1 : 0;
  }
}

// Copy from pinned host memory (mapped into the device address space).
__global__ void fetch_kernel(double* __restrict__ dst, const double* __restrict__ src, long long n) {
  for (long long i = blockIdx.x * (long long)blockDim.x + threadIdx.x; i < n; i += (long long)gridDim.x * blockDim.x)
    dst[i] = src[i];
}

// ---------------------------------------------------------------------------
// Launchers
// ---------------------------------------------------------------------------
namespace {
inline int cdiv(long long a, long long b) { return (int)((a + b - 1) / b); }
}  // namespace

int launch_fetch(void* dst, const void* src, size_t bytes, void* stream) {
  const long long n = (long long)(bytes / sizeof(double));
  if (n <= 0) return hipSuccess;
  const int nb = (int)std::max<long long>(1, std::min<long long>(512, (n + 255) / 256));
  PHIQ_LAUNCH(fetch_kernel, dim3(nb), dim3(256), 0, (hipStream_t)stream, (double*)dst, (const double*)src, n);
  return hipGetLastError();
}

int launch_gemm_jobs(const GemmJob* jobs, int njobs, int nmax, void* stream, const int* stop) {
  if (njobs <= 0) return hipSuccess;
  if (nmax <= kPanelK) {
    dim3 grid(cdiv(nmax, 32), cdiv(nmax, 32), njobs);
    PHIQ_LAUNCH(gemm_panel_kernel, grid, dim3(256), 0, (hipStream_t)stream, jobs, stop);
    return hipGetLastError();
  }
  // few large-tile blocks would leave most CUs idle: use one-wave 32x32 tiles
  if ((long long)njobs * cdiv(nmax, 64) * cdiv(nmax, 64) < 512) {
    using C = Tile32;
    dim3 grid(cdiv(nmax, C::BM), cdiv(nmax, C::BN), njobs);
    PHIQ_LAUNCH(gemm_jobs_kernel<C>, grid, dim3(C::NT), 0, (hipStream_t)stream, jobs, stop);
  } else {
    using C = Tile64;
    dim3 grid(cdiv(nmax, C::BM), cdiv(nmax, C::BN), njobs);
    PHIQ_LAUNCH(gemm_jobs_kernel<C>, grid, dim3(C::NT), 0, (hipStream_t)stream, jobs, stop);
  }
  return hipGetLastError();
}

int launch_scale_jobs(const ScaleJob* jobs, int njobs, int nmax, void* stream, const int* stop) {
  if (njobs <= 0) return hipSuccess;
  dim3 grid(std::max(1, std::min(64, cdiv((long long)nmax * nmax, 256))), njobs);
  PHIQ_LAUNCH(scale_jobs_kernel, grid, dim3(256), 0, (hipStream_t)stream, jobs, stop);
  return hipGetLastError();
}

int launch_taylor_jobs(const TaylorJob* jobs, int njobs, int nmax, void* stream, const int* stop) {
  if (njobs <= 0) return hipSuccess;
  dim3 grid(std::max(1, std::min(64, cdiv((long long)nmax * nmax, 256))), njobs);
  PHIQ_LAUNCH(taylor_jobs_kernel, grid, dim3(256), 0, (hipStream_t)stream, jobs, stop);
  return hipGetLastError();
}

namespace {
inline int outer(const TtmArgs& a) { return a.nouter > 1 ? a.nouter : 1; }
// several right-hand sides in one launch: only the FP64 rotated kernels
inline bool two_index(const TtmArgs& a) { return a.emod > 0 || a.xdiv > 0 || a.nouter > 1 || a.seg.n > 0; }

template <class C>
dim3 ttm_grid(const TtmArgs& a, int nb) {
  const long long T = ttm_tiles<C>(a.M, a.L, nb);
  return dim3((unsigned)(((T + kXcds - 1) / kXcds) * kXcds), 1, 1);
}

// 16-byte vector loads need even row lengths and 16-byte aligned operands
// (natural layout: X rows have L elements)
bool vec_ok(const TtmArgs& a) {
  uintptr_t ptrs = (uintptr_t)a.E | (uintptr_t)a.X;
  for (int s = 0; s < a.seg.n && s < kSegMax; ++s) ptrs |= (uintptr_t)a.seg.sx[s];
  return (a.K % 2 == 0) && (!a.nn || a.L % 2 == 0) && (ptrs % 16 == 0) && (a.es % 2 == 0) && (a.xs % 2 == 0) &&
         (a.xo % 2 == 0);
}

template <class C>
int store_cfg(const TtmArgs& a, hipStream_t st) {
  if (vec_ok(a))
    PHIQ_LAUNCH((ttm_store_kernel<C, true>), ttm_grid<C>(a, a.nbatch), dim3(C::NT), 0, st, a);
  else
    PHIQ_LAUNCH((ttm_store_kernel<C, false>), ttm_grid<C>(a, a.nbatch), dim3(C::NT), 0, st, a);
  return hipGetLastError();
}
template <class C>
int square_cfg(const TtmArgs& a, hipStream_t st) {
  if (vec_ok(a))
    PHIQ_LAUNCH((ttm_square_kernel<C, true>), ttm_grid<C>(a, a.nbatch * outer(a)), dim3(C::NT), 0, st, a);
  else
    PHIQ_LAUNCH((ttm_square_kernel<C, false>), ttm_grid<C>(a, a.nbatch * outer(a)), dim3(C::NT), 0, st, a);
  return hipGetLastError();
}
template <class C, bool VEC>
int accum_np(const TtmArgs& a, hipStream_t st) {
  const dim3 g = ttm_grid<C>(a, outer(a));
  switch (a.np) {
    case 1: PHIQ_LAUNCH((ttm_accum_kernel<C, 1, VEC>), g, dim3(C::NT), 0, st, a); break;
    case 2: PHIQ_LAUNCH((ttm_accum_kernel<C, 2, VEC>), g, dim3(C::NT), 0, st, a); break;
    case 3: PHIQ_LAUNCH((ttm_accum_kernel<C, 3, VEC>), g, dim3(C::NT), 0, st, a); break;
    default: PHIQ_LAUNCH((ttm_accum_kernel<C, 4, VEC>), g, dim3(C::NT), 0, st, a); break;
  }
  return hipGetLastError();
}
template <class C>
int accum_cfg(const TtmArgs& a, hipStream_t st) {
  return vec_ok(a) ? accum_np<C, true>(a, st) : accum_np<C, false>(a, st);
}

// Last product after the slab product (X in its natural layout): fixed
// shapes, those the autotuner picks for the rotated kernels at n = 128.
template <class C>
int store_nn(const TtmArgs& a, hipStream_t st) {
  if (vec_ok(a))
    PHIQ_LAUNCH((ttm_store_kernel<C, true, true>), ttm_grid<C>(a, a.nbatch), dim3(C::NT), 0, st, a);
  else
    PHIQ_LAUNCH((ttm_store_kernel<C, false, true>), ttm_grid<C>(a, a.nbatch), dim3(C::NT), 0, st, a);
  return hipGetLastError();
}
template <class C, bool VEC>
int accum_nn_v(const TtmArgs& a, hipStream_t st) {
  static_assert(C::BM == Tile64p1w8::BM && C::BN == Tile64p1w8::BN && C::NT == Tile64p1w8::NT, "same grid");
  const dim3 g = ttm_grid<C>(a, outer(a));
  switch (a.np) {
    case 1: PHIQ_LAUNCH((ttm_accum_kernel<C, 1, VEC, true>), g, dim3(C::NT), 0, st, a); break;
    case 2: PHIQ_LAUNCH((ttm_accum_kernel<C, 2, VEC, true>), g, dim3(C::NT), 0, st, a); break;
    case 3: PHIQ_LAUNCH((ttm_accum_kernel<C, 3, VEC, true>), g, dim3(C::NT), 0, st, a); break;
    // four running sums do not fit in 128 registers
    default: PHIQ_LAUNCH((ttm_accum_kernel<Tile64p1w8, 4, VEC, true>), g, dim3(C::NT), 0, st, a); break;
  }
  return hipGetLastError();
}
template <class C>
int square_nn(const TtmArgs& a, hipStream_t st) {
  if (vec_ok(a))
    PHIQ_LAUNCH((ttm_square_kernel<C, true, true>), ttm_grid<C>(a, a.nbatch * outer(a)), dim3(C::NT), 0, st, a);
  else
    PHIQ_LAUNCH((ttm_square_kernel<C, false, true>), ttm_grid<C>(a, a.nbatch * outer(a)), dim3(C::NT), 0, st, a);
  return hipGetLastError();
}
template <class C, bool VEC>
int square_all_nn_v(const TtmArgs& a, hipStream_t st) {
  const dim3 g = ttm_grid<C>(a, outer(a));
  switch (a.nbatch) {
    case 1: PHIQ_LAUNCH((ttm_square_all_kernel<C, 1, VEC, true>), g, dim3(C::NT), 0, st, a); break;
    case 2: PHIQ_LAUNCH((ttm_square_all_kernel<C, 2, VEC, true>), g, dim3(C::NT), 0, st, a); break;
    case 3: PHIQ_LAUNCH((ttm_square_all_kernel<C, 3, VEC, true>), g, dim3(C::NT), 0, st, a); break;
    default: PHIQ_LAUNCH((ttm_square_all_kernel<Tile64p1w8, 4, VEC, true>), g, dim3(C::NT), 0, st, a); break;
  }
  return hipGetLastError();
}
int launch_nn(int kind, const TtmArgs& a, hipStream_t st) {
  const bool v = vec_ok(a);
  if (kind == 1) return v ? accum_nn_v<Tile64p1w8m2, true>(a, st) : accum_nn_v<Tile64p1w8m2, false>(a, st);
  if (kind == 2) {
    if (a.order0 != 0 || a.yacc || a.nbatch > 4 || a.es != 0) return square_nn<Tile64x128>(a, st);
    return v ? square_all_nn_v<Tile64p1w8m2, true>(a, st) : square_all_nn_v<Tile64p1w8m2, false>(a, st);
  }
  // too few 64 x 128 tiles to fill the GPU three blocks per CU: 64 x 64, 32-deep chunks
  return ttm_tiles<Tile64x128p1w8>(a.M, a.L, a.nbatch) < 768 ? store_nn<Tile64k32>(a, st)
                                                              : store_nn<Tile64x128p1w8>(a, st);
}

// default tile choice when no tuned entry exists (from sweeps on gfx950 at
// n = 32, 128, 256: 64 x 128 tiles for the stores, 64 x 64 with 32-deep K
// chunks for small n, for the node sum and, with all orders per block, for
// the squaring step)
int default_cfg(int kind, int M, int nb) {
  if (kind == 1) return 3;
  if (kind == 2) return nb <= 4 ? 8 : 0;  // all orders per block when p <= 4
  return M >= 128 ? 5 : 6;
}
}  // namespace

int ttm_num_configs(int kind) { return kind == 1 ? 7 : (kind == 2 ? 12 : 14); }

int launch_ttm_store(const TtmArgs& a, phiq_precision prec, void* stream, int cfg) {
  if (two_index(a) && prec != PHIQ_PREC_FP64) return hipErrorInvalidValue;
  if (prec == PHIQ_PREC_BF16X3 && !a.nn) {
    const int r = launch_ttm_store_bf16r(a, stream, cfg);
    if (r != hipErrorNotSupported) return r;
  }
  if (prec == PHIQ_PREC_FP32 && !a.nn) {
    const int r = launch_ttm_store_f32r(a, stream, cfg);
    if (r != hipErrorNotSupported) return r;
  }
  if (prec != PHIQ_PREC_FP64) return a.nn ? hipErrorInvalidValue : launch_ttm_store_lowp(a, prec, stream);
  hipStream_t st = (hipStream_t)stream;
  if (a.nn) return launch_nn(0, a, st);
  if (cfg < 0) cfg = default_cfg(0, a.M, a.nbatch);
  switch (cfg) {
    case 0: return store_cfg<Tile64>(a, st);
    case 1: return store_cfg<Tile128>(a, st);
    case 2: return store_cfg<Tile128x128>(a, st);
    case 3: return store_cfg<Tile256>(a, st);
    case 4: return store_cfg<Tile128k32>(a, st);
    case 5: return store_cfg<Tile64x128>(a, st);
    case 6: return store_cfg<Tile64k32>(a, st);
    case 7: return store_cfg<Tile128x128w8>(a, st);
    case 8: return store_cfg<Tile64x128p1>(a, st);
    case 9: return store_cfg<Tile128p1>(a, st);
    case 10: return store_cfg<Tile64p1>(a, st);
    case 11: return store_cfg<Tile64x128p1w8>(a, st);
    case 12: return store_cfg<Tile128p1w8>(a, st);
    case 13: return store_cfg<Tile128x128p1>(a, st);
  }
  return hipErrorInvalidValue;
}

int launch_ttm_accum(const TtmArgs& a, phiq_precision prec, void* stream, int cfg) {
  if (two_index(a) && prec != PHIQ_PREC_FP64) return hipErrorInvalidValue;
  if (a.np > 4 || a.np < 1) return hipErrorInvalidValue;
  if (prec != PHIQ_PREC_FP64) return a.nn ? hipErrorInvalidValue : launch_ttm_accum_lowp(a, prec, stream);
  hipStream_t st = (hipStream_t)stream;
  if (a.nn) return launch_nn(1, a, st);
  if (cfg < 0) cfg = default_cfg(1, a.M, a.nbatch);
  switch (cfg) {
    case 0: return accum_cfg<Tile64>(a, st);
    case 1: return accum_cfg<Tile128>(a, st);
    case 2: return accum_cfg<Tile64x128>(a, st);
    case 3: return accum_cfg<Tile64k32>(a, st);
    case 4: return accum_cfg<Tile64x128p1r>(a, st);
    case 5: return accum_cfg<Tile64p1>(a, st);
    case 6: return accum_cfg<Tile64p1w8>(a, st);
  }
  return hipErrorInvalidValue;
}

namespace {
template <class C, bool VEC>
int square_all_np(const TtmArgs& a, hipStream_t st) {
  const dim3 g = ttm_grid<C>(a, outer(a));
  switch (a.nbatch) {
    case 1: PHIQ_LAUNCH((ttm_square_all_kernel<C, 1, VEC>), g, dim3(C::NT), 0, st, a); break;
    case 2: PHIQ_LAUNCH((ttm_square_all_kernel<C, 2, VEC>), g, dim3(C::NT), 0, st, a); break;
    case 3: PHIQ_LAUNCH((ttm_square_all_kernel<C, 3, VEC>), g, dim3(C::NT), 0, st, a); break;
    default: PHIQ_LAUNCH((ttm_square_all_kernel<C, 4, VEC>), g, dim3(C::NT), 0, st, a); break;
  }
  return hipGetLastError();
}
template <class C>
int square_all_cfg(const TtmArgs& a, hipStream_t st) {
  return vec_ok(a) ? square_all_np<C, true>(a, st) : square_all_np<C, false>(a, st);
}
}  // namespace

int launch_ttm_square(const TtmArgs& a, phiq_precision prec, void* stream, int cfg) {
  if (two_index(a) && prec != PHIQ_PREC_FP64) return hipErrorInvalidValue;
  if (prec == PHIQ_PREC_BF16X3 && !a.nn) {
    const int r = launch_ttm_square_bf16r(a, stream, cfg);
    if (r != hipErrorNotSupported) return r;
  }
  if (prec == PHIQ_PREC_FP32 && !a.nn) {
    const int r = launch_ttm_square_f32r(a, stream, cfg);
    if (r != hipErrorNotSupported) return r;
  }
  if (prec != PHIQ_PREC_FP64) return a.nn ? hipErrorInvalidValue : launch_ttm_square_lowp(a, prec, stream);
  hipStream_t st = (hipStream_t)stream;
  if (a.nn) return launch_nn(2, a, st);
  // an order offset or an accumulating store needs the per-order kernel:
  // 64 x 128 tiles when they fill the GPU twice over, else 64 x 64 (the last
  // step of a linear combination is one vector: 64 x 128 tiles left one
  // four-wave block per CU)
  if ((a.order0 != 0 || a.yacc) && (cfg < 0 || cfg >= 7))
    cfg = (a.M >= 128 && ttm_tiles<Tile64x128>(a.M, a.L, a.nbatch * outer(a)) >= 768) ? 5 : 6;
  if (cfg < 0) cfg = default_cfg(2, a.M, a.nbatch);
  // shapes 7.. : all orders per block (p <= 4)
  if (cfg >= 7) {
    if (a.nbatch > 4 || a.es != 0) return hipErrorInvalidValue;
    switch (cfg) {
      case 7: return square_all_cfg<Tile64>(a, st);
      case 8: return square_all_cfg<Tile64k32>(a, st);
      case 9: return square_all_cfg<Tile128>(a, st);
      case 10: return square_all_cfg<Tile64p1>(a, st);
      case 11: return square_all_cfg<Tile64p1w8>(a, st);
    }
    return hipErrorInvalidValue;
  }
  switch (cfg) {
    case 0: return square_cfg<Tile64>(a, st);
    case 1: return square_cfg<Tile128>(a, st);
    case 2: return square_cfg<Tile128x128>(a, st);
    case 3: return square_cfg<Tile256>(a, st);
    case 4: return square_cfg<Tile128k32>(a, st);
    case 5: return square_cfg<Tile64x128>(a, st);
    case 6: return square_cfg<Tile64k32>(a, st);
  }
  return hipErrorInvalidValue;
}

int launch_absdiff_max(const double* y, const double* yold, int np, long long N, double* partial, int nblocks,
                       void* stream, const int* stop) {
  PHIQ_LAUNCH(absdiff_max_kernel, dim3(nblocks), dim3(256), 0, (hipStream_t)stream, y, yold, np, N, partial, stop);
  return hipGetLastError();
}

int launch_cc_decide(const double* partial, int nblk, int np, double tol, const int* prev, CcCtl* out,
                     void* stream) {
  PHIQ_LAUNCH(cc_decide_kernel, dim3(1), dim3(256), 0, (hipStream_t)stream, partial, nblk, np, tol, prev, out);
  return hipGetLastError();
}

int launch_node_sum(const NodeSegs& segs, long long N, const double* coef, int ldcoef, int np, double* Y,
                    void* stream, const int* stop) {
  const int nb = std::max(1, std::min(4096, cdiv(N, 256)));
  switch (np) {
    case 1: PHIQ_LAUNCH(node_sum_kernel<1>, dim3(nb), dim3(256), 0, (hipStream_t)stream, segs, N, coef, ldcoef, np, Y, stop); break;
    case 2: PHIQ_LAUNCH(node_sum_kernel<2>, dim3(nb), dim3(256), 0, (hipStream_t)stream, segs, N, coef, ldcoef, np, Y, stop); break;
    case 3: PHIQ_LAUNCH(node_sum_kernel<3>, dim3(nb), dim3(256), 0, (hipStream_t)stream, segs, N, coef, ldcoef, np, Y, stop); break;
    case 4: PHIQ_LAUNCH(node_sum_kernel<4>, dim3(nb), dim3(256), 0, (hipStream_t)stream, segs, N, coef, ldcoef, np, Y, stop); break;
    default: PHIQ_LAUNCH(node_sum_kernel<0>, dim3(nb), dim3(256), 0, (hipStream_t)stream, segs, N, coef, ldcoef, np, Y, stop);
  }
  return hipGetLastError();
}

}  // namespace phiq
