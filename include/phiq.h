/*
 * phiq.h -- phi-function actions of Kronecker-sum matrices on AMD MI355X.
 *
 * Computes  out[k] = phi_k(-t A) v,  k = 0..p,  for
 *     A = A^0 (+) A^1 (+) ... (+) A^{D-1}
 *       = sum_d I (x) .. (x) A^d (x) .. (x) I        (Section 2.2, eq. KronA)
 * with phi_0(M) = e^M and phi_k(M) = int_0^1 e^{(1-s)M} s^{k-1}/(k-1)! ds
 * (Section 2.1, eq. Varphi), by the quadrature + scaling and modified
 * squaring method of Croci & Munoz-Matute (Section 3, Algorithms 1, 2 and
 * phiquadmv, eq. squaring).  Only 1D exponentials of the n_d x n_d factors
 * are formed; they are applied to v viewed as an n_0 x n_1 (x n_2) tensor by
 * mode products (eq. Expkron, eq. KronAb).
 *
 * Conventions shared by every entry point
 *   * Tensor layout: v and each out[k] are row-major tensors of shape
 *     (n_0, n_1, ..., n_{D-1}), axis 0 slowest; A^d acts on axis d (this is
 *     the order of the Kronecker products in eq. KronA).  N = prod_d n_d.
 *   * Matrices: A^d is n_d x n_d, row-major, FP64.
 *   * Pointers marked HOST are ordinary host memory; pointers marked DEVICE
 *     are device memory of the handle's GPU (e.g. from hipMalloc or a torch
 *     CUDA tensor).  The caller owns every pointer it passes; the library
 *     never frees or keeps them after the call returns (plans keep device
 *     copies of what they need).
 *   * Streams: device work is enqueued on the given hipStream_t (0 = the
 *     legacy default stream) and is asynchronous unless stated otherwise;
 *     the caller must keep inputs alive and outputs untouched until the
 *     stream reaches that point.
 *   * Errors: every call returns a phiq_status.  Arguments are validated on
 *     the host before any device work is enqueued; on an error nothing is
 *     enqueued and output buffers are left unchanged, except where noted.
 *     No C++ exception crosses this boundary.
 *   * Threads: a handle may be used from one host thread at a time.
 */
#ifndef PHIQ_H
#define PHIQ_H

#include <stddef.h>
#include <stdint.h>
#include <hip/hip_runtime_api.h>

#ifdef __cplusplus
extern "C" {
#endif

#define PHIQ_MAX_DIM 4
#define PHIQ_MAX_P 24
#define PHIQ_MAX_N 1024

typedef enum {
  PHIQ_OK = 0,
  PHIQ_ERR_INVALID_ARG = -1,   /* a size, pointer or option out of range      */
  PHIQ_ERR_NONFINITE = -2,     /* t, tol or an entry of A^d is not finite     */
  PHIQ_ERR_NOT_CONVERGED = -3, /* adaptive Clenshaw-Curtis hit its cap        */
  PHIQ_ERR_OOM = -4,           /* device allocation failed or over the cap    */
  PHIQ_ERR_HIP = -5,           /* a HIP runtime call failed                   */
  PHIQ_ERR_UNSUPPORTED = -6    /* valid request the library does not implement */
} phiq_status;

/* Quadrature rule of the integral form (the `type` input of phiquadmv):
 * fixed Gauss-Legendre with the node count of the a priori bound
 * (Algorithm 1), or adaptive nested Clenshaw-Curtis (Algorithm 2). */
typedef enum { PHIQ_RULE_GAUSS = 1, PHIQ_RULE_CC = 2 } phiq_rule;

/* Arithmetic of the mode products.  The 1D exponentials, the node sums and
 * the squaring recurrence are always FP64. */
typedef enum {
  PHIQ_PREC_FP64 = 0,    /* FP64 MFMA, FP64 intermediates                    */
  PHIQ_PREC_FP32 = 1,    /* FP32 MFMA with FP32 accumulation                 */
  PHIQ_PREC_BF16X3 = 2,  /* x = hi + lo in bf16, hi*hi + hi*lo + lo*hi, FP32 */
  PHIQ_PREC_INT8 = 3     /* FP64 split into S signed 7-bit digits (5 for tol  */
                         /* >= 1e-6, 6 for >= 1e-9, else 7) with one exponent */
                         /* per row of a 1D factor and per tensor; digit      */
                         /* products exact on int8 MFMA, combined in FP64.    */
                         /* Gauss rule, dim >= 2, every n_d in {32, 64, 96,  */
                         /* 128} (else PHIQ_ERR_UNSUPPORTED).               */
} phiq_precision;

/* Scaling l of adaptive Clenshaw-Curtis (Algorithm 2). */
typedef enum {
  PHIQ_CC_SCALING_REALIZED = 0, /* least predicted cost of the nodes Algorithm 2 */
                                /* will run (phiq_cc_scaling)                    */
  PHIQ_CC_SCALING_PAPER = 1     /* Algorithm setup_quadrature with the CC bound  */
} phiq_cc_scaling_mode;

/* Choice of (l, m) for the Gauss rule. */
typedef enum { PHIQ_SEL_PAPER = 0, PHIQ_SEL_MLP = 1, PHIQ_SEL_MLP_EMPIRICAL = 2 } phiq_selector;

/* The Kronecker-sum operator: D = dim factors, HOST pointers. */
typedef struct {
  int dim;                        /* 1..PHIQ_MAX_DIM                          */
  int n[PHIQ_MAX_DIM];            /* n_d in 1..PHIQ_MAX_N                     */
  const double* A[PHIQ_MAX_DIM];  /* HOST, n_d x n_d row-major FP64           */
} phiq_kron_op;

typedef struct {
  phiq_rule rule;           /* default PHIQ_RULE_GAUSS                              */
  phiq_precision precision; /* default PHIQ_PREC_FP64                               */
  int l;                    /* scaling exponent; -1 = choose (setup_quadrature)     */
  int m;                    /* Gauss node count (n+1); -1 = choose; CC ignores it  */
  double alpha;             /* estimate of ||tA||_inf; < 0 = eq. infnorm_upper_bnd  */
  double c1, c2;            /* cost model C = c1 d n + c2 (n + l p); default 0, 1   */
  int cc_max_doublings;     /* cap of Algorithm 2's doubling loop; default 6        */
  size_t workspace_cap;     /* device bytes the handle may hold; 0 = no cap         */
  int use_graphs;           /* phiq_action, Gauss rule: 1 = from the third call of  */
                            /* one shape on, replay the device work from a captured */
                            /* hipGraph (bitwise the same result).  Default 0: on   */
                            /* ROCm 7 a replay of the ~45-node graph costs more     */
                            /* than the eager launches it replaces.                 */
  int selector;             /* Gauss (l, m) choice when l and m are not forced:     */
                            /* PHIQ_SEL_PAPER (default, Algorithm setup_quadrature),*/
                            /* PHIQ_SEL_MLP (the handle's network, certified: its   */
                            /* outputs are l and m, the bound of Thm 3.2 judges the */
                            /* pair; see phiq_selector_set) or                      */
                            /* PHIQ_SEL_MLP_EMPIRICAL (the network's outputs are l  */
                            /* and log10 rho, rho in [0.1, 1]: m is Algorithm       */
                            /* quadnodes at the norm rho ||tA|| and scaling l, rho  */
                            /* learned from measured errors of the method's own     */
                            /* sweeps, so the bound at ||tA|| does not certify the  */
                            /* result; only for tol >= 1e-10, below which           */
                            /* Algorithm setup_quadrature chooses).  A network      */
                            /* choice costing over 1.5x Algorithm                   */
                            /* setup_quadrature's in chain count (m + l p) is       */
                            /* rejected in both modes.                              */
  int slab_products;        /* FP64, three axes with n_1 = n_2 = 128: the products  */
                            /* along axes 2 and 1 in one pass per 128 x 128 slab    */
                            /* (the same sums, the k-loops associated otherwise)    */
                            /* for 1 chains of one vector (phi_0, single terms of a */
                            /* combination), 2 every chain, 0 none (default: on     */
                            /* gfx950 at n = 128 it saved no time in a phi-action   */
                            /* and cost 3% in ETD-RK4)                              */
  int accept_floor;         /* FP32 / BF16X3: 0 (default) = a tol below the form's  */
                            /* rounding floor (PHIQ_FLOOR_FP32 / _BF16X3) is        */
                            /* refused with PHIQ_ERR_UNSUPPORTED; 1 = run anyway:   */
                            /* the result then carries the floor, not tol, and the  */
                            /* report says so (precision_floor, tol_met = 0)        */
  double selector_slack;    /* PHIQ_SEL_MLP: decades by which the a priori bound at */
                            /* the network's (l, m) may exceed tol (0..12).  0, the */
                            /* default, is the certified mode: the bound must meet  */
                            /* tol, as in Algorithm setup_quadrature                */
  int batch_persistent;     /* phiq_action_batched: 1 = the whole batch in one      */
                            /* persistent launch (tiles handed out in dependency    */
                            /* order, workgroups waiting on per-group completion    */
                            /* counters); the call then waits for the launch and    */
                            /* returns PHIQ_ERR_HIP if a wait gave up (bounded,     */
                            /* seconds).  0 (default) = one launch per dependency   */
                            /* depth, asynchronous                                  */
  int rhs_per_launch;       /* phiq_plan_execute, Gauss rule, FP64, no slab         */
                            /* products: right-hand sides that share each mode-     */
                            /* product launch (node, vector) as one batch index.    */
                            /* 0 (default) = as many as fit in PHIQ_RHS_GROUP_BYTES */
                            /* of intermediates; 1 = one vector at a time; k = at   */
                            /* most k.  Same sums: bitwise the same when the same   */
                            /* kernels run (the kernel can depend on the launch's   */
                            /* size: at n_d = 256 large plain products sum k in     */
                            /* another order, see phiq_tile_config kind 5).  1 also */
                            /* keeps the vectors of phiq_plan_execute_combo in      */
                            /* separate launches (otherwise, FP64 Gauss with every  */
                            /* b_1..b_p set and p <= 4, all node chains and phi_0's */
                            /* chain share one launch per mode product and one node */
                            /* sum: the same sums, another rounding order)          */
  int cc_scaling;           /* PHIQ_RULE_CC: PHIQ_CC_SCALING_REALIZED (default) or  */
                            /* PHIQ_CC_SCALING_PAPER; the accuracy is the stopping  */
                            /* test's either way                                    */
} phiq_options;

/* Device bytes of intermediates a group of right-hand sides may take when
 * they share launches (rhs_per_launch = 0). */
#define PHIQ_RHS_GROUP_BYTES ((size_t)8 << 30)

/* Rounding floors of the lower-precision mode products: an upper level of
 * the relative error per phi_k (inf-norm, against the exact action) that
 * the FP32-accumulated products leave whatever the quadrature and squaring
 * do, measured on the 3D advection-diffusion workloads up to n_d = 256
 * (FP32 ~8e-7, split bf16 ~9e-6) with a margin.  The method's own
 * truncation error (log10_bound) comes on top of it. */
#define PHIQ_FLOOR_FP32 2e-6
#define PHIQ_FLOOR_BF16X3 3e-5

/* What a plan / call did.  Times are filled by phiq_action only. */
typedef struct {
  int l;               /* scaling exponent used                                 */
  int m;               /* quadrature nodes used (n+1)                           */
  int cc_doublings;    /* doublings of Algorithm 2 (0 for Gauss)                */
  int ttm_chains;      /* applications of a Kronecker product of 1D factors     */
  double alpha;        /* ||tA||_inf estimate used by the selector              */
  double log10_bound;  /* log10 of the a priori bound at (l, m), relative to ||v||_inf */
  double cc_err;       /* last relative change of Algorithm 2 (0 for Gauss)     */
  size_t workspace_bytes; /* device bytes held by the handle after the call     */
  int selector;        /* how (l, m) was chosen: 0 Algorithm setup_quadrature   */
                       /* (or forced), 1 network, 2 network with m raised to    */
                       /* what the bound needs, 3 network rejected (fallback),  */
                       /* 4 empirical-mode network (PHIQ_SEL_MLP_EMPIRICAL)     */
  double precision_floor; /* rounding floor of the mode products' precision     */
                       /* (PHIQ_FLOOR_FP32 / _BF16X3; 0 for FP64 and int8       */
                       /* digits, whose digit count follows tol)                */
  int tol_met;         /* 1 if tol >= precision_floor, i.e. the requested       */
                       /* tolerance is within what the precision form reaches;  */
                       /* 0 only when accept_floor let a smaller tol through    */
} phiq_report;

typedef struct phiq_handle_s* phiq_handle;
typedef struct phiq_plan_s* phiq_plan;

/* Status name, e.g. "PHIQ_ERR_INVALID_ARG".  Never NULL. */
const char* phiq_status_string(phiq_status s);

/* Defaults: Gauss, FP64, choose l and m, alpha from eq. infnorm_upper_bnd,
 * c1 = 0, c2 = 1 (the values used in Section 4), cc cap 6, no workspace cap. */
phiq_status phiq_options_default(phiq_options* opt);

/* ---------------------------------------------------------------------------
 * Host-only planning (no GPU needed).
 * ------------------------------------------------------------------------ */

/* alpha = |t| * sum_d ||A^d||_inf, the upper bound eq. infnorm_upper_bnd. */
phiq_status phiq_norm_bound(const phiq_kron_op* op, double t, double* alpha);

/* Parameter selection, Algorithms quaderr / quadnodes / setup_quadrature
 * (Section 3.2-3.3) with the a priori bound of Thm 3.2, for the largest
 * order p, tolerance eps, norm estimate alpha and vector factor beta.
 * rule selects which bound (Gauss or Clenshaw-Curtis) is used.  Outputs:
 * *l, *n (the paper's n: the rule has n+1 nodes) and *cost = C(n, l, p).
 * d is the spatial dimension entering c1 d n.  p = 0 gives l = 0, n = -1. */
phiq_status phiq_setup_quadrature(double eps, int p, double alpha, double beta,
                                  phiq_rule rule, double c1, double c2, int d,
                                  int* l, int* n, double* cost);

/* Scaling of adaptive Clenshaw-Curtis by the cost of the nodes Algorithm 2
 * will run (the plan's default, PHIQ_CC_SCALING_REALIZED).  Algorithm 2
 * stops about one nested level (7, 13, 25, ... points) after the first rule
 * that is accurate.  For each l in [l_paper - 1, l_paper + 3] (l_paper from
 * Algorithm setup_quadrature with the CC bound), the first accurate level is
 * predicted with the CC bound of Thm 3.2 at alpha / 4, and the l with the
 * least C = c1 d n + c2 (n + l p) over the nodes run (n + 1) is returned;
 * ties keep the smaller l.  The a priori bound at alpha, not alpha / 4, is
 * what certifies the paper's l; here accuracy comes from Algorithm 2's
 * stopping test. */
phiq_status phiq_cc_scaling(double eps, int p, double alpha, double c1, double c2, int d,
                            int max_doublings, int* l);

/* log of Algorithm quaderr: max over q = 1..p of the Thm 3.2 bound for the
 * (n+1)-node rule at norm alpha and vector factor beta.  n may be real. */
phiq_status phiq_log_quaderr(double n, int p, double alpha, double beta,
                             phiq_rule rule, double* log_err);

/* Algorithm quadnodes: the smallest n (the rule has n+1 nodes) whose
 * Thm 3.2 bound at norm alpha and vector factor beta is <= eps, for orders
 * 1..p (root of the bound in n, rounded up; n >= 2 Gauss, >= 4 CC). */
phiq_status phiq_quadnodes(double eps, int p, double alpha, double beta, phiq_rule rule, int* n);

/* Nodes theta and weights w on [0, 1] of the m-point Gauss-Legendre rule
 * (rule = GAUSS) or the m-point Clenshaw-Curtis rule (rule = CC, m >= 2,
 * nodes theta_j = (1 + cos(j pi/(m-1)))/2, j = 0..m-1).  HOST arrays of m. */
phiq_status phiq_quadrature_rule(phiq_rule rule, int m, double* theta, double* w);

/* ---------------------------------------------------------------------------
 * Device entry points.
 * ------------------------------------------------------------------------ */

/* Create a handle bound to HIP device `device` (made current during calls).
 * The handle owns a growable device workspace that later calls reuse, so
 * repeated calls of the same size allocate nothing. */
phiq_status phiq_create(phiq_handle* h, int device);
phiq_status phiq_destroy(phiq_handle h);  /* synchronises the device, frees all */

/* Plan: validates, estimates alpha, selects (l, m) (Gauss) or l (CC) with
 * tolerance tol read relative to ||v||_inf (the bound is linear in
 * ||b||_inf, so beta = 1), builds the rule, uploads A^d and forms on the
 * GPU every 1D exponential the plan needs:
 *   exp((1 - theta_q) 2^{-l} (-t A^d)) for each node q,
 *   exp(2^{k-l} (-t A^d)) for k = 0..l (squaring factors and phi_0).
 * The exponentials are enqueued on `stream`.  opt may be NULL (defaults).
 * rep may be NULL. */
phiq_status phiq_plan_create(phiq_handle h, const phiq_kron_op* op, double t, int p,
                             double tol, const phiq_options* opt, phiq_plan* plan,
                             phiq_report* rep, hipStream_t stream);

/* Execute a plan on nrhs vectors: v DEVICE nrhs x N, out DEVICE
 * nrhs x (p+1) x N (out[r][k] = phi_k(-tA) v[r]).  v and out must not
 * overlap.  Gauss plans run asynchronously and allocate nothing once the
 * handle's workspace is large enough; with FP64 products the vectors of a
 * group (opt.rhs_per_launch) share every launch: one per mode product for
 * all their node chains, one node sum, one phi_0 product and one per
 * squaring product, so the workspace grows with the group.  Clenshaw-Curtis
 * plans read the convergence decision of each level back to the host
 * (Algorithm 2).  rep may be NULL. */
phiq_status phiq_plan_execute(phiq_plan plan, const double* v, int nrhs, double* out,
                              phiq_report* rep, hipStream_t stream);

/* out = sum_{j=0}^{p} phi_j(-tA) b_j for the plan's (A, t, p): one linear
 * combination of the phi-functions against p+1 different vectors (the
 * remark on linear combinations after Algorithm 2, which gives the one-pass
 * quadrature of sum_{j>=1} phi_j b_j without scaling).  Here it is combined
 * with scaling and squaring: the node sums of all b_j feed p scaled
 * intermediates that obey eq. squaring, so the cost is p chains per node,
 * p per squaring step (one in the last) and one for b_0, instead of
 * (m + l j + 1) chains per vector for separate phi-actions.
 *   b    HOST array of p+1 DEVICE pointers, b[j] -> N doubles (tensor layout
 *        as for phiq_action); NULL entries are zero vectors, at least one
 *        entry must be non-NULL.  out DEVICE N doubles, must not overlap any
 *        b[j].
 *   With a Clenshaw-Curtis plan, Algorithm 2's doubling runs on the p scaled
 *   intermediates: every level's node vectors of every b_j are kept, and the
 *   doubling stops when the largest relative change of the intermediates is
 *   below the tolerance (one stream synchronisation per doubling, as in
 *   phiq_plan_execute; PHIQ_ERR_NOT_CONVERGED at the plan's doubling cap).
 *   Errors: PHIQ_ERR_INVALID_ARG (NULL plan/b/out, all b[j] NULL, overlap),
 *   PHIQ_ERR_UNSUPPORTED (int8-digit plans, or l (p-1) > 900, which would
 *   overflow the 2^{l (p-j)} factors), PHIQ_ERR_NOT_CONVERGED.  FP32 and
 *   split-bf16 plans run their mode products in that form, the node sums and
 *   squaring in FP64, as phiq_plan_execute does.
 * Accuracy (Gauss): the plan's bound holds for each term, so the error is at
 * most tol * sum_j ||b_j||_inf plus rounding.  Gauss plans run
 * asynchronously on `stream`; both use the handle's workspace like
 * phiq_plan_execute. */
phiq_status phiq_plan_execute_combo(phiq_plan plan, const double* const* b, double* out,
                                    hipStream_t stream);

phiq_status phiq_plan_destroy(phiq_plan plan);

/* For callers that cannot allocate device memory: code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc.  Runs
 * phiq_plan_execute for one vector (nrhs = 1) of a Gauss-rule plan with
 * FP64, FP32 or split-bf16 mode products, keeping its intermediate tensors in
 * a fixed device array of the library instead of the handle's workspace.  It
 * allocates and frees nothing; the plan (phiq_plan_create) and v, out are
 * the caller's.
 *   v     DEVICE, N doubles; out DEVICE, (p+1) x N doubles; no overlap.
 *   need  HOST, nullable: set to the bytes of the array the plan needs,
 *         2 max(m+1, p) N e + 2 p N 8 (e = 8 for FP64, 4 otherwise; each
 *         term rounded up to 256), also when that exceeds the array.
 * The array holds PHIQ_NOALLOC_SCRATCH_BYTES (64 MiB) per GPU, from the
 * library's load until the process ends.  Errors: PHIQ_ERR_OOM when the plan
 * needs more than that (e.g. 3D n = 64 with m <= 12 fits, n = 128 does not);
 * PHIQ_ERR_UNSUPPORTED for the Clenshaw-Curtis rule, int8 digits, or while
 * live timing (phiq_profile_start) is on.  No element of the array needs to
 * start at zero: the call reads only what it wrote first.  Every call on one
 * GPU shares that GPU's array and leaves its contents behind: calls that
 * overlap on one GPU (other streams, threads or handles) race and must be
 * ordered by the caller. */
#define PHIQ_NOALLOC_SCRATCH_BYTES ((size_t)64 << 20)
phiq_status phiq_plan_execute_noalloc(phiq_plan plan, const double* v, double* out, size_t* need,
                                      hipStream_t stream);

/* One call: plan_create + plan_execute + plan_destroy.  v DEVICE N,
 * out DEVICE (p+1) x N.  The whole call is on `stream`; the host returns
 * after enqueueing (Gauss) or after the last error check (CC). */
phiq_status phiq_action(phiq_handle h, const phiq_kron_op* op, double t, int p,
                        const double* v, double tol, const phiq_options* opt,
                        double* out, phiq_report* rep, hipStream_t stream);

/* One problem of a batch: operator, time, order, tolerance and nrhs vectors
 * that share them (e.g. the stage vectors of an exponential Runge-Kutta
 * step).  A[d] HOST as for phiq_action; v DEVICE nrhs x N; out DEVICE
 * nrhs x (p+1) x N.  rep (nullable) receives l, m, alpha, the bound and
 * ttm_chains summed over the problem's vectors. */
typedef struct {
  phiq_kron_op op;
  double t;
  int p;
  double tol;
  int nrhs;
  const double* v;
  double* out;
  phiq_report* rep;
} phiq_problem;

/* Many independent phi-actions (Algorithm 6 per problem) launched together.
 * Every problem gets the parameters phiq_action would choose with the same
 * options (so the results agree with separate calls up to the summation
 * order of the tiles).  Problems with the Gauss rule, FP64 mode products and
 * p <= 4 are split into stages (1D exponentials, node chains with the node
 * sum, squaring steps, phi_0), and the stages of all of them are run by
 * depth in their dependency graph: one kernel launch per depth and stage
 * type covers those tiles of every problem, so small and large problems fill
 * the GPU together (a batch of 512 mixed 2D/3D problems takes ~62 depths).
 * Other problems (CC, lower precision, p > 4) run afterwards, one plan each,
 * on the same stream (then the call synchronises the stream).  Asynchronous
 * otherwise.  Device memory: the handle keeps one arena for the batch
 * (factors and the per-vector workspaces of all problems, ~16 N doubles per
 * vector plus the 1D matrices); opt->workspace_cap bounds it (PHIQ_ERR_OOM).
 * Outputs must not overlap each other or any v (inputs may be shared). */
phiq_status phiq_action_batched(phiq_handle h, int nprob, const phiq_problem* probs,
                                const phiq_options* opt, hipStream_t stream);

/* Host-only dry run of phiq_action_batched's scheduling (no GPU needed; v
 * and out are only compared as addresses): validates the problems exactly
 * as the batched call does, builds the stage list and checks that every
 * address a stage touches lies in the arena or in its problem's v / out and
 * that every stage runs at a greater depth than the stages it reads. */
typedef struct {
  int persistent;          /* problems in the persistent launch          */
  int separate;            /* problems run one plan each afterwards      */
  long long stages;        /* stages of the persistent launch            */
  long long tiles;         /* work items (64 x 64 tiles) over all stages */
  int depth;               /* longest dependency chain, in stages        */
  int launches;            /* kernel launches (one per depth and stage type) */
  int groups;              /* dependency groups                          */
  size_t arena_bytes;      /* device bytes the handle's batch arena needs */
  size_t upload_bytes;     /* host->device bytes per call                 */
} phiq_batch_stats;
phiq_status phiq_batch_info(int nprob, const phiq_problem* probs, const phiq_options* opt,
                            phiq_batch_stats* info);

/* Exponential time differencing of order four (Cox and Matthews' ETD-RK4,
 * the paper's reference cox2002exponential; Section 5 runs lower-order
 * exponential integrators on the same phi-function actions) for
 *   u' = -A u + c1 u + c3 u^3,   A = sum_d A^d as for phiq_action,
 * nsteps steps of size tau, in place on u (DEVICE, N values).  Each step uses
 * e^{-tau A/2}, phi_1(-tau A/2), e^{-tau A} and phi_1..3(-tau A), tolerance
 * tol relative to the vector's max norm, plans built once per call.
 * form 0: four plans; phi_0..p of every stage vector, the last plan on three
 * vectors in one execution; work buffer 27 N doubles.  form 1: every stage
 * is one phiq_plan_execute_combo (two plans, about 30% fewer mode products
 * at p = 3); work buffer 11 N doubles.
 * use_graph = 1: the first step runs directly, the second is captured into a
 * hipGraph (on a stream of the call's own) and replayed for every later step.
 * Returns when the steps have finished.  rep (nullable) gets the plans and
 * how the steps ran. */
typedef struct {
  int steps_eager;          /* steps launched directly                      */
  int steps_graph;          /* steps replayed from the captured graph       */
  int graph_nodes;          /* nodes (kernels) of one captured step         */
  int ttm_chains_per_step;  /* Kronecker chains of 1D factors per step      */
  int l_half, m_half;       /* plan of phi_0..1(-tau A/2)                   */
  int l_full, m_full;       /* plan of phi_0..3(-tau A)                     */
} phiq_etd_report;
phiq_status phiq_etdrk4(phiq_handle h, const phiq_kron_op* op, double tau, int nsteps,
                        double c1, double c3, double tol, int use_graph, int form, double* u,
                        phiq_etd_report* rep, hipStream_t stream);

/* The exponential Runge-Kutta methods of Section 5 (Table RK) on the paper's
 * Problem 3 (Hochbruck-Ostermann): u' = -A u + 1/(1 + u^2) + f(x, y, t) on
 * (0,1)^2 with A = A^0 (+) A^1 (dim 2, n x n interior grid, nodes
 * x_i = (i+1)/(n+1), x slowest) and f the manufactured source for which
 * u = x(1-x) y(1-y) e^t solves the PDE.  method 1 = exponential Euler,
 * 2 = RK2 with c2, 3 = RK3 with c2 and c3 = 2/3.  nsteps steps of T/nsteps
 * from t = 0, in place on u (DEVICE n^2 values, the initial condition on
 * entry).  phi-actions with tolerance tol and options opt (rule etc.).
 * form 0: the vectors of one stage go through one plan execution (phi_0..p
 * of each, then combined); allocates 13 n^2 doubles.  form 1: every stage
 * is one phiq_plan_execute_combo (not with int8-digit plans:
 * PHIQ_ERR_UNSUPPORTED), about half the mode products; allocates 6 n^2
 * doubles.  Returns when the steps have finished.  rep (nullable): the
 * full-step plan.  PHIQ_ERR_UNSUPPORTED for other dimensions. */
phiq_status phiq_exprk(phiq_handle h, const phiq_kron_op* op, int method, double c2, int nsteps,
                       double T, double tol, const phiq_options* opt, int form, double* u,
                       phiq_report* rep, hipStream_t stream);

/* ---------------------------------------------------------------------------
 * Learned (l, m) selector: a network 8 -> 64 -> 64 -> 2 with tanh hidden
 * layers in FP32.  Parameters, one vector of PHIQ_MLP_NPARAM floats: W1
 * (64 x 8, row-major), b1 (64), W2 (64 x 64), b2 (64), W3 (2 x 64), b3 (2).
 * Inputs (8): log10 t||A^d||_inf for axes 0..2 (-3 for an absent axis),
 * max_d n_d / 256, dim, p, log10 t, log10 tol; outputs: l / 8 and m / 16
 * (PHIQ_SEL_MLP), or l / 8 and log10 rho (PHIQ_SEL_MLP_EMPIRICAL).
 * Loss: mean of (y - target)^2 over the B x 2 outputs.
 * ------------------------------------------------------------------------ */
#define PHIQ_MLP_NPARAM 4866

/* Y = net(X): X DEVICE B x 8, w DEVICE PHIQ_MLP_NPARAM, Y DEVICE B x 2. */
phiq_status phiq_mlp_forward(phiq_handle h, int B, const float* X, const float* w, float* Y,
                             hipStream_t stream);
/* Gradient of the loss at w (DEVICE grad, PHIQ_MLP_NPARAM), summed over the
 * samples in a fixed order; *loss (HOST, nullable) = the loss.  T DEVICE
 * B x 2 targets.  Synchronises the stream when loss is requested. */
phiq_status phiq_mlp_grad(phiq_handle h, int B, const float* X, const float* T, const float* w,
                          float* grad, double* loss, hipStream_t stream);
/* Full-batch Adam (beta1 0.9, beta2 0.999, eps 1e-8) for `steps` steps from
 * the HOST weights w (updated in place), HOST data X (B x 8) and T (B x 2);
 * loss_history (HOST, nullable) gets the loss before each step.  Blocks. */
phiq_status phiq_mlp_train(phiq_handle h, int B, const float* X, const float* T, float* w, int steps,
                           float lr, float* loss_history);
/* The handle's selector network (HOST w copied; NULL clears it). */
phiq_status phiq_selector_set(phiq_handle h, const float* w);
/* The same from a file: exactly PHIQ_MLP_NPARAM little-endian IEEE float32
 * values, in the order of the parameter vector above (weights_path HOST,
 * NUL-terminated).  PHIQ_ERR_INVALID_ARG if the file cannot be opened or
 * holds another number of bytes, PHIQ_ERR_NONFINITE for a NaN or infinite
 * weight; the handle's network is unchanged on error. */
phiq_status phiq_selector_load(phiq_handle h, const char* weights_path);

/* Building blocks (also used by the tests).
 *
 * phiq_expm: E[b] = exp(X[b]) for nmat matrices n x n, DEVICE row-major
 * FP64, by truncated Taylor series with scaling and squaring (the same
 * kernels the plans use).  xnorm HOST[nmat]: an upper bound on ||X[b]||_inf
 * (selects the scaling).  X and E must not overlap.
 *
 * phiq_kron_apply: y[r] = (F^0 (x) F^1 (x) ... (x) F^{D-1}) x[r] for nvec
 * vectors, F DEVICE pointers (HOST array of D pointers to n_d x n_d
 * row-major FP64), x and y DEVICE nvec x N, not overlapping. */
phiq_status phiq_expm(phiq_handle h, int n, int nmat, const double* X, const double* xnorm,
                      double* E, hipStream_t stream);
phiq_status phiq_kron_apply(phiq_handle h, int dim, const int* n, const double* const* F,
                            const double* x, double* y, int nvec, phiq_precision prec,
                            hipStream_t stream);

/* ---------------------------------------------------------------------------
 * Live kernel timing.
 *
 * Between phiq_profile_start and phiq_profile_stop the handle brackets every
 * kernel it launches with a pair of HIP events on the launch stream.  stop
 * synchronises the device and returns, per kernel class, the number of
 * launches, the summed event time and the algorithmic work of those
 * launches: flops of the contractions (2 n N per mode product of one
 * N-vector) and the bytes each launch must move at least (every operand
 * read once, every result written once).  Classes: "ttm_store",
 * "ttm_accum", "ttm_square", "gemm", "taylor", "scale", "node_sum",
 * "absdiff".  stats is HOST, room for max_stats entries; *n_stats gets the
 * number of classes with at least one launch.
 * ------------------------------------------------------------------------ */
typedef struct {
  char name[24];
  int launches;
  double ms;       /* summed event time of the launches                   */
  double flops;    /* algorithmic floating-point operations               */
  double bytes;    /* algorithmic bytes (compulsory reads + writes)       */
} phiq_kernel_stat;

/* class_mask: bit c set = bracket launches of class c (order above:
 * bit 0 ttm_store, 1 ttm_accum, 2 ttm_square, 3 gemm, 4 taylor, 5 scale,
 * 6 node_sum, 7 absdiff); 0 = all classes.  Each bracket adds a little
 * time to the stream, so timing only the classes of interest keeps the
 * rest of the work undisturbed. */
phiq_status phiq_profile_start(phiq_handle h, unsigned class_mask);
phiq_status phiq_profile_stop(phiq_handle h, phiq_kernel_stat* stats, int max_stats, int* n_stats);

/* Pause (on = 0) or resume (on != 0) the bracketing that phiq_profile_start
 * began, keeping the launches recorded so far and the class mask; no device
 * work, no synchronisation.  A bracketed launch leaves the GPU idle for a
 * few microseconds around it, so timing a sample of a long run's launches
 * disturbs its throughput less than timing every one.  INVALID_ARG if h is
 * NULL or no profile is open (before phiq_profile_start or after stop). */
phiq_status phiq_profile_enable(phiq_handle h, int on);

/* Tile shape of the mode products for every later launch of one kind:
 * FP64 kind 0 (plain mode product), 1 (with the node sum), 2 (with the
 * squaring combination); split bf16 and FP32 kind 3 (plain) and 4
 * (squaring), where cfg 0 is the general tile kernel and cfg >= 1 the
 * kernels that keep the 1D factor resident in LDS (split bf16: n_d in {64,
 * 128, 256}, store cfg 1..5, squaring 1..2; FP32: n_d in {128, 256}, store
 * cfg 1..3, squaring 1..2 with FP32 input; other shapes and cfgs take the
 * general kernel); FP64 with the factor resident in LDS, kind 5
 * (plain), 6 (squaring), 7 (node sum): cfg 0 declines (the tile kernels of
 * kinds 0..2 run), cfg >= 1 forces a resident shape for the launches it
 * takes (n_d in {64, 128, 256}, FP64 in and out), -1 = default (kinds 5
 * and 6 resident at n_d = 256 when the launch fills the GPU; kind 7 off:
 * it measured slower than the tile kernel).  A forced shape of kinds 0..2
 * also turns the resident kernels off for that kind.  cfg -1 restores the
 * autotuned or default choice, 0..count-1 forces that shape (tuning,
 * testing; FP64 squaring shapes 7.. need p <= 4).  *count (nullable) =
 * number of shapes of the kind. */
phiq_status phiq_tile_config(phiq_handle h, int kind, int cfg, int* count);

/* ---------------------------------------------------------------------------
 * Autotuner.
 *
 * Times every tile shape of the FP64 mode-product kernels on the launch
 * shapes a phi-action with these sizes makes (dim axes of sizes n[d], p
 * orders, m quadrature nodes: node products with m + 1 batches (the Gauss
 * nodes and phi_0's chain), phi_0's last product with 1,
 * squaring products with p batches, the fused node sum and the fused
 * squaring step)
 * and keeps the fastest shape per launch shape in the handle; later calls
 * with those shapes use it.  Synchronises the stream.  times may be NULL or
 * HOST [64][16]: row r = launch shape r in the order above, column c = the
 * time in ms of tile shape c (rows and columns that do not exist are left
 * untouched).  The workspace contents are overwritten.
 * ------------------------------------------------------------------------ */
phiq_status phiq_autotune(phiq_handle h, int dim, const int* n, int p, int m, double* times,
                          hipStream_t stream);

#ifdef __cplusplus
}
#endif
#endif /* PHIQ_H */
