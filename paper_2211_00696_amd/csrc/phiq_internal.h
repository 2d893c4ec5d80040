// Internal declarations shared by the library's translation units.
#pragma once

#include <cstddef>
#include <cstdint>

#include "phiq.h"

namespace phiq {

// Start/stop events for the next kernel launch (live timing): when set, the
// launchers attach them to the kernel's own dispatch (hipExtLaunchKernel),
// so no separate event packets enter the stream.
extern thread_local void* g_launch_events[2];

// ---- planner.cpp ----------------------------------------------------------
void poly_coeffs(double n, int p, double alpha, phiq_rule rule, double* a3, double* a2, double* a1);
double log_bound_at(double rho, double n, int p, double alpha, double beta, phiq_rule rule);
double best_log_bound(double n, int p, double alpha, double beta, phiq_rule rule);
double log_quaderr(double n, int p, double alpha, double beta, phiq_rule rule);
int quadnodes(double eps, int p, double alpha, double beta, phiq_rule rule);
void setup_quadrature(double eps, int p, double alpha, double beta, phiq_rule rule, double c1,
                      double c2, int d, int* l, int* n, double* cost);
// Adaptive Clenshaw-Curtis: the scaling with the least predicted cost of
// Algorithm 2's realized node count (l_paper: Algorithm setup_quadrature's).
int cc_scaling(double eps, int p, double alpha, double c1, double c2, int d, int max_doublings, int l_paper);
void gauss_legendre(int m, double* theta, double* w);
void clenshaw_curtis(int m, double* theta, double* w);

// ---- api.cpp --------------------------------------------------------------
phiq_status validate_op(const phiq_kron_op* op);
// noalloc.hip: resolve the fixed scratch array's address on `device` (which
// must be current); api.cpp: one Gauss execution with a caller workspace.
phiq_status noalloc_scratch_init(int device);
phiq_status plan_execute_in(phiq_plan P, const double* v, double* out, void* ws, size_t ws_cap, hipStream_t st,
                            size_t* need);
int plan_device(phiq_plan P);
// Rounding floor of a precision form's mode products (0 where the digit
// count or FP64 follows tol).
inline double precision_floor(phiq_precision prec) {
  return prec == PHIQ_PREC_FP32 ? PHIQ_FLOOR_FP32 : prec == PHIQ_PREC_BF16X3 ? PHIQ_FLOOR_BF16X3 : 0.0;
}
double sum_infnorms(const phiq_kron_op* op);

// Host-chosen parameters of one phi-action (Algorithm setup_quadrature with beta = 1).
struct PlanParams {
  double alpha;        // ||tA||_inf estimate
  double log10_bound;  // a priori quadrature bound at (l, m)
  int l;               // scaling exponent
  int m;               // Gauss nodes (0 for CC or p = 0)
  int K;               // Taylor degree of the 1D exponentials
  int sigma[PHIQ_MAX_DIM];  // extra halvings of axis d's Taylor argument
  int selector;        // phiq_report::selector
};
// mlp: the handle's selector network (nullable).
phiq_status select_params(const phiq_kron_op* op, double t, int p, double tol, const phiq_options& opt,
                          PlanParams* pp, const float* mlp);
const float* handle_mlp(phiq_handle h);  // the handle's selector network or null

// ---- mlp.hip / mlp.cpp: the selector network ------------------------------
constexpr int kMlpIn = 8, kMlpHidden = 64, kMlpOut = 2;
constexpr int kMlpParams = kMlpHidden * kMlpIn + kMlpHidden + kMlpHidden * kMlpHidden + kMlpHidden +
                           kMlpOut * kMlpHidden + kMlpOut;
int launch_mlp_forward(const float* w, const float* X, int B, float* H1, float* H2, float* Y, void* stream);
int launch_mlp_backward(const float* w, const float* T, const float* H1, const float* H2, const float* Y, int B,
                        float* dY, float* dZ2, float* dZ1, double* loss_part, void* stream);
int launch_mlp_wgrad(const float* X, const float* H1, const float* H2, const float* dZ1, const float* dZ2,
                     const float* dY, int B, int chunks, double* part, float* grad, void* stream);
int launch_mlp_adam(float* w, const float* g, float* m, float* v, float lr, float b1, float b2, float eps, int step,
                    void* stream);
// Host forward pass (the same arithmetic as the kernel) and the planner's
// use of it: features, prediction, the bound as judge.  Returns false when
// the prediction is rejected (the caller keeps Algorithm setup_quadrature's choice).
void mlp_predict_host(const float* w, const float x[kMlpIn], float y[kMlpOut]);
// slack: factor by which the bound at the network's choice may exceed tol
// (1 = certified mode).
bool mlp_choose(const float* w, const phiq_kron_op* op, const double* norms, double t, int p, double tol,
                double slack, double alpha, int l5, int n5, int* l, int* n, int* used);
// Empirical mode (PHIQ_SEL_MLP_EMPIRICAL): the network's outputs are l / 8 and
// log10 of the norm ratio at which the a priori bound covered the measured
// errors of the method's own sweeps; n is Algorithm quadnodes at that norm
// and scaling l.  Declines (used 0) below kEmpiricalTolMin, the smallest
// tolerance the sweeps covered; used 4 = the network's pair, 3 = rejected.
constexpr double kEmpiricalTolMin = 1e-10;
bool mlp_choose_empirical(const float* w, const phiq_kron_op* op, const double* norms, double t, int p,
                          double tol, double alpha, int l5, int n5, int* l, int* n, int* used);
// Grow-only device arena of batched calls, held by the handle.
phiq_status batch_arena(phiq_handle h, size_t bytes, void** dev);
// Pinned staging slot of at least `bytes`, and its upload (a copy kernel
// reading the pinned memory, on st).
phiq_status batch_stage(phiq_handle h, size_t bytes, int* slot, void** host);
phiq_status batch_fetch(phiq_handle h, int slot, void* dst, size_t bytes, hipStream_t st);
// Wait until the plan's own device work (1D exponentials) has finished and
// stop its executions from waiting on it: after this, execution enqueues
// only kernels on the caller's stream (what a stream capture needs).
phiq_status plan_settle(phiq_plan P);
bool plan_profiling(phiq_plan P);  // live kernel timing is on for the plan's handle

// ---- exprk.hip: Problem 3 of Section 5 ---------------------------------------
// g = g(t, e + sa a + sb b) with g(t, u) = 1/(1+u^2) + f(x, y, t) on the n x n
// interior grid of (0,1)^2 (a, b nullable); copy (nullable) = e.
int launch_exprk_stage(const double* e, const double* a, double sa, const double* b, double sb, int n, double t,
                       double* g, double* copy, void* stream);
// out = x + sa a + sb b (a, b nullable); out may alias x or a
int launch_exprk_comb(const double* x, const double* a, double sa, const double* b, double sb, double* out,
                      long long N, void* stream);
// out = sa a + sb b (b may be null)
int launch_exprk_axpby(const double* a, double sa, const double* b, double sb, double* out, long long N,
                       void* stream);

// ---- etd.hip: elementwise steps of the ETD-RK4 integrator ----------------
// F(x) = c1 x + c3 x^3.  All arrays DEVICE, n elements.
int launch_etd_nonlin(const double* x, double* fx, long long n, double c1, double c3, void* stream);
// a = x + s y; fa = F(a) (a may be null: not stored)
int launch_etd_stage(const double* x, const double* y, double s, double* a, double* fa, long long n, double c1,
                     double c3, void* stream);
// b = x + s y; fb = F(b); mix = 2 fb - fu; sum = fa + fb
int launch_etd_stage_b(const double* x, const double* y, double s, const double* fu, const double* fa, double* mix,
                       double* sum, long long n, double c1, double c3, void* stream);
// u = e + h [(g1_1 - 3 g1_2 + 4 g1_3) + 2 (g2_2 - 2 g2_3) + (-g3_2 + 4 g3_3)], gr_k = g + (4 r + k) n
int launch_etd_final(const double* e, const double* g, double h, double* u, long long n, void* stream);
// linear-combination form: fx = F(x), s = hs fx
int launch_etd_cf_stage(const double* x, double* fx, double* s, double hs, long long n, double c1, double c3,
                        void* stream);
// s = hs (2 F(b) - fu), fab = fa + F(b)
int launch_etd_cf_b(const double* b, const double* fu, const double* fa, double* s, double* fab, double hs,
                    long long n, double c1, double c3, void* stream);
// the phi_1..3 vectors of the final update from F(u), F(a) + F(b) and c
int launch_etd_cf_final(const double* c, const double* fu, const double* fab, double* b1, double* b2, double* b3,
                        double h, long long n, double c1, double c3, void* stream);
int launch_etd_copy(const double* x, double* y, long long n, void* stream);

// ---- kernels.hip: device job descriptors ---------------------------------
// C = A * B, all n x n row-major FP64 (A, B, C distinct).
struct GemmJob {
  const double* A;
  const double* B;
  double* C;
  int n;
  int pad_;
};

// out = s * src, n x n.
struct ScaleJob {
  const double* src;
  double* dst;
  double s;
  int n;
  int pad_;
};

// dst[t] = sum_{k=0}^{K} c[t]^k/k! Z^k, t < nt, with Z^0 = I and Z^k stored at
// Zpow + (k-1) n^2 for k = 1..K (truncated Taylor series of exp(c Z)); the
// powers are read once per element for all nt coefficients.
constexpr int kTaylorTargets = 16;
constexpr int kMaxTaylorDegree = 32;
struct TaylorJob {
  const double* Zpow;
  double* dst[kTaylorTargets];
  double c[kTaylorTargets];
  int n;
  int K;
  int nt;
};

// Mode product of a row-major (L x K) tensor view X with the M x K matrix
// E (M = K = n_d), written rotated: out[i' * L + j] = sum_k E[i'][k] X[j][k].
// Applying it once per axis, last axis first, returns the tensor to its
// original layout after D steps.  Batch b uses E + b*es, X + b*xs, O + b*os.
// X and O are FP64 for the FP64 path; with a lower precision the
// intermediate tensors between mode products are FP32 (x_f32 / o_f32 say
// which side is FP32; strides are in elements).  With nn set (FP64 only)
// X is read in its natural layout instead, X[k * L + j]: the last product
// after the two-axis slab product, which leaves the layout unchanged.
// Batch segments of a plain FP64 product: batches [sb[s], sb[s+1]) take
// factor se[s] + (b - sb[s]) and, when sx[s] is set, the one input vector
// sx[s] (the first product of the node chains of several vectors of a
// linear combination, plus phi_0's factor for b_0).
constexpr int kSegMax = 5;
struct TtmSegs {
  int n;
  int sb[kSegMax + 1];
  int se[kSegMax];
  const double* sx[kSegMax];
};

struct TtmArgs {
  const double* E;
  long long es;
  // lower precision: the same matrices converted (FP32 in Ea, or bf16 hi in
  // Ea and lo in Eb), element-indexed like E
  const void* Ea;
  const void* Eb;
  const void* X;
  long long xs;
  void* O;
  long long os;
  int x_f32, o_f32;
  int nn;
  int M, K, L, nbatch;
  // node-sum epilogue: Y + j*ys = sum_b 2^cexp coef[j * ldcoef + b] * C_b, j < np
  const double* coef;
  int ldcoef;
  int np;
  int cexp;
  double* Y;
  long long ys;
  // squaring epilogue: batch b is order i = b + 1 + order0;
  // O_b = 2^{-i} (C_b + sum_{j=1}^{i} (Yprev + (j-1)*yps)/(i-j)!)
  const double* Yprev;
  long long yps;
  int order0;
  // node sum and per-order squaring (FP64): 1 = add the result to Y / O
  int yacc;
  // nullable: a device flag; when it is set the launch does nothing (the
  // speculative level of adaptive Clenshaw-Curtis after convergence)
  const int* stop;
  // Several right-hand sides in one launch (FP64 rotated kernels only).
  // Plain products: when emod > 0 batch b takes factor b % emod, and when
  // xdiv > 0 input b / xdiv (the node chains of several vectors, b = r *
  // emod + i for vector r and node i: emod in every product, xdiv in the
  // first, which reads the vectors themselves).  Node sum and
  // squaring: nouter > 1 independent problems r, each offset by r * xo in X,
  // r * yo in Y, r * oo in O and r * ypo in Yprev.
  int emod, xdiv;
  int nouter;
  long long xo, yo, oo, ypo;
  TtmSegs seg;  // n = 0: none (plain products only; emod and xdiv unused)
  double ifact[PHIQ_MAX_P + 1];  // ifact[k] = 1/k!
};

// Host launchers (kernels.hip).  All return hipSuccess or the launch error.
// dst (device) = src (pinned host memory, read by the kernel), bytes % 8 == 0
int launch_fetch(void* dst, const void* src, size_t bytes, void* stream);
int launch_gemm_jobs(const GemmJob* jobs_dev, int njobs, int nmax, void* stream, const int* stop = nullptr);
int launch_scale_jobs(const ScaleJob* jobs_dev, int njobs, int nmax, void* stream, const int* stop = nullptr);
int launch_taylor_jobs(const TaylorJob* jobs_dev, int njobs, int nmax, void* stream, const int* stop = nullptr);
// cfg selects the FP64 tile shape (-1: default); kinds 0 = store, 1 = node
// sum, 2 = squaring; ttm_num_configs(kind) shapes exist per kind.
int ttm_num_configs(int kind);
int launch_ttm_store(const TtmArgs& a, phiq_precision prec, void* stream, int cfg);
int launch_ttm_accum(const TtmArgs& a, phiq_precision prec, void* stream, int cfg);
int launch_ttm_square(const TtmArgs& a, phiq_precision prec, void* stream, int cfg);
// Split-bf16 products with the factor resident in LDS (kernels_bf16r.hip),
// n in {64, 128, 256}: hipErrorNotSupported for other shapes or cfg 0 (the
// caller then runs the general kernel).  Store cfg 1..3 pick the wave and
// column-block shape, -1 the default.
int bf16r_num_configs();
int bf16r_square_num_configs();
int launch_ttm_store_bf16r(const TtmArgs& a, void* stream, int cfg);
// FP64 with the factor resident in LDS (kernels_f64r.hip): n in {64, 128,
// 256}; cfg 0 declines, -1 = default; hipErrorNotSupported when declined
int launch_ttm_store_f64r(const TtmArgs& a, void* stream, int cfg);
int launch_ttm_square_f64r(const TtmArgs& a, void* stream, int cfg);
int launch_ttm_accum_f64r(const TtmArgs& a, void* stream, int cfg);
int f64r_num_configs();
int f64r_accum_num_configs();
int launch_ttm_square_bf16r(const TtmArgs& a, void* stream, int cfg);
// FP32 with the factor resident in LDS (kernels_f32r.hip): n in {128, 256},
// the FP32 twin of E; store cfg 1..3, squaring cfg 1..2 (FP32 X), 0
// declines, -1 = default; hipErrorNotSupported when declined
int launch_ttm_store_f32r(const TtmArgs& a, void* stream, int cfg);
int launch_ttm_square_f32r(const TtmArgs& a, void* stream, int cfg);

// Products along axes 2 and 1 of nbatch tensors n0 x kSlabN x kSlabN in one
// pass (kernels_slab.hip), layout unchanged:
//   O_b[i0][j1][j2] = sum_{k1,k2} E1_b[j1][k1] E2_b[j2][k2] X_b[i0][k1][k2],
// batch b at X + b*xs, E1 + b*es1, E2 + b*es2, O + b*os (FP64; X, E1, E2
// 16-byte aligned, strides even).
constexpr int kSlabN = 128;
struct SlabArgs {
  const double* X;
  long long xs;
  const double* E1;
  long long es1;
  const double* E2;
  long long es2;
  double* O;
  long long os;
  int n0, nbatch;
};
bool slab2_supported(const SlabArgs& a);
int launch_slab2(const SlabArgs& a, void* stream);
// FP32-MFMA and split-bf16 (3-product) versions (kernels_lowp.hip)
// dst = src converted to FP32 (a) or split into bf16 hi (a) and lo (b)
int launch_convert(const double* src, long long count, phiq_precision prec, void* a, void* b, void* stream,
                   const int* stop = nullptr);
int launch_ttm_store_lowp(const TtmArgs& a, phiq_precision prec, void* stream);
int launch_ttm_accum_lowp(const TtmArgs& a, phiq_precision prec, void* stream);
int launch_ttm_square_lowp(const TtmArgs& a, phiq_precision prec, void* stream);

// CC error: partial maxima of |y_j - yold_j| and |y_j| over blocks.
// partial[(blk * np + j) * 2 + {0, 1}] = block maxima of |y_j - yold_j|, |y_j|
// with y_j = y + j*N, yold_j = yold + j*N.
int launch_absdiff_max(const double* y, const double* yold, int np, long long N, double* partial,
                       int nblocks, void* stream, const int* stop = nullptr);
// Convergence test of Algorithm 2 on the device: err = max_j max_b num / max_b
// den over the partial maxima of nblk blocks; stop = (prev && *prev) || err <= tol.
struct CcCtl {
  double err;
  int stop;
  int pad_;
};
int launch_cc_decide(const double* partial, int nblk, int np, double tol, const int* prev, CcCtl* out,
                     void* stream);
// Node vectors stored in up to 12 segments (one per adaptive level).
struct NodeSegs {
  const double* V[12];
  int count[12];
  int nseg;
};
// Y + j*N = sum_b coef[j * ldcoef + b] * V_b, nodes numbered through the
// segments in order.
int launch_node_sum(const NodeSegs& segs, long long N, const double* coef, int ldcoef, int np, double* Y,
                    void* stream, const int* stop = nullptr);

// ---- kernels_i8.hip: mode products on int8 digit slices -------------------
enum I8Mode : int { kI8Slice = 0, kI8Store = 1, kI8Square = 2 };
struct I8Args {
  int S;                                // digits per value (5..7)
  const int8_t* E;                      // factor digits: batch b at E + b es, slice s at + s esp
  long long es, esp;                    // rows of K digits, M rows per factor
  const int* ee;                        // row exponents: batch b at ee + b ees
  long long ees;
  int delta;                            // 2^delta bounds ||E_b||_inf (digit epilogue)
  const int8_t* X;                      // input digits: batch b at X + b xs, slice s at + s xsp
  long long xs, xsp;
  const int* xe;                        // input tensor exponent of batch b: xe[b xes]
  long long xes;
  int M, K;
  long long L;
  int nbatch;
  int8_t* O8;                           // kI8Slice: output digits O8 + b os8 + s osp8
  long long os8, osp8;
  int* oe;                              // kI8Slice: output exponents, oe[b] = xe + delta
  double* O;                            // kI8Store / kI8Square: O + b os
  long long os;
  const double* Yprev;                  // kI8Square: y_j at Yprev + (j-1) yps; batch b is order b+1
  long long yps;
  double ifact[PHIQ_MAX_P + 1];
};
// digits of the rows of X (rows x K, contiguous) with one exponent per row
int launch_i8_slice_rows(const double* X, long long rows, int K, int S, int8_t* planes, int* ex, void* stream);
// digits of nt tensors X + r xs (N values each) with one exponent per
// tensor (partial: nt x nbx doubles of scratch); planes + r bstride, ex[r]
int launch_i8_slice_tensors(const double* X, long long xs, long long N, int nt, int S, double* partial, int nbx,
                            int8_t* planes, long long bstride, int* ex, void* stream);
// M = K in {32, 64, 96, 128}, L % 32 == 0
int launch_i8_product(const I8Args& a, int mode, void* stream);

// ---- batched.hip: batched stages, one launch per dependency depth --------
// A batch is a list of stages (one GEMM, Taylor evaluation or mode product
// over a whole operand, split into 64 x 64 tiles), stored by depth in the
// dependency graph (then by type, order count and staging width); tiles are
// numbered consecutively over the list.  One launch runs the tiles of one
// such kind at one depth.  `signal`/`wait*` record the
// dependencies for the host-side check of the order.
enum BatchStageType : int {
  kStageGemm = 0,    // O = E * X (n x n, n = M)
  kStageTaylor = 1,  // Taylor sums of job `aux` (BatchTaylor)
  kStageStore = 2,   // O_b = rotated mode product of (E_b, X_b), b < nb
  kStageAccum = 3,   // Y_q (+)= sum_b coef[q * ldcoef + b] * (E_b X_b), q < np
  kStageSquare = 4,  // O_i = 2^{-i-1} (E X_i + sum_{j<=i} Y_j / (i-j)!), i < np
  kStageStoreWide = 5,   // as kStageStore with 64 x 128 tiles and 512 threads (M >= kBatchWideM)
  kStageAccumWide = 6,   // as kStageAccum, 512 threads (8 waves of 32 x 16) on the same 64 x 64 tiles (M >= kBatchWaves8M)
  kStageSquareWide = 7,  // as kStageSquare, likewise
};
struct BatchStage {
  long long tile0;  // number of this stage's first tile
  int ntiles;
  int type;
  int signal;       // dependency group this stage belongs to
  int wait0, need0; // groups whose results it reads (-1: none) and their tile counts
  int wait1, need1;
  int M, K, L, nb;
  int np;
  int vec;          // 16-byte staging allowed (K even, 16-byte aligned E and X)
  int accumulate;   // Accum: add into Y
  int ldcoef;
  int aux;          // Taylor: job index
  int pad_;
  const double* E;
  long long es;
  const double* X;
  long long xs;
  double* O;
  long long os;
  const double* coef;
  double* Y;
  long long ys;
};
// dst[t] = I + sum_{k=1}^{K} c[t]^k/k! Z^k (t < nt), Z^1 at Z1 and Z^k at
// Zp + (k-2) n^2 for k >= 2.
struct BatchTaylor {
  const double* Z1;
  const double* Zp;
  double* dst[kTaylorTargets];
  double c[kTaylorTargets];
  int n;
  int K;
  int nt;
  int pad_;
};
constexpr int kBatchTile = 64;          // output tile edge of every stage (rows of a wide store tile)
constexpr int kBatchWideN = 128;        // columns of a wide store tile
constexpr int kBatchWideM = 96;         // stores with at least this many rows use wide tiles
constexpr int kBatchWaves8M = 64;       // node sums / squaring steps from this many rows use eight waves
constexpr int kBatchTaylorChunk = 4096; // elements per Taylor tile
struct BatchArgs {
  const BatchStage* st;
  int stage_begin;       // stages [stage_begin, stage_end) of one launch (one depth, one type)
  int stage_end;
  long long tile_begin;  // their tiles [tile_begin, tile_end)
  long long tile_end;
  const BatchTaylor* tj;
};
// One launch over the tiles of a run of stages with the same type, np
// (Accum, Square) and vec; blocks must be a multiple of 8.
int launch_batch(const BatchArgs& a, int type, int np, int vec, int blocks, void* stream);
// The whole batch in one persistent launch (batched.hip): tiles handed out
// from ctl->next in the schedule's order; done[g] counts the finished tiles
// of group g; a wait that polls spin_limit times sets ctl->err and ends.
struct BatchPersistCtl {
  unsigned long long next;
  int err;
  int pad_;
};
struct BatchPersistArgs {
  BatchPersistCtl* ctl;
  unsigned* done;
  long long total;       // tiles of the schedule
  int nstages;
  int pad_;
  long long spin_limit;  // polls per wait before giving up
};
int launch_batch_persistent(const BatchArgs& a, const BatchPersistArgs& p, void* stream);

}  // namespace phiq
