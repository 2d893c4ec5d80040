// C ABI: handles, plans and execution of the phi-action
// (Algorithms 1, 2 and phiquadmv of Croci & Munoz-Matute, Section 3).
//
// Device work per plan (all on the caller's stream):
//   plan:    upload A^d; Z_d = -t 2^{-l-sigma_d} A^d; powers Z_d^2..Z_d^K;
//            exp(c Z_d) by the truncated Taylor series for every node
//            coefficient c = 1 - theta_q and for c = 1; sigma_d squarings;
//            l more squarings give exp(2^{k-l}(-t A^d)), k = 1..l.
//   execute: for every node, the Kronecker product of its 1D exponentials
//            applied to v (D mode products, last axis first, written
//            rotated so the tensor returns to its layout), with the node
//            sum fused into the last product; then l modified-squaring steps
//            (eq. squaring), each D mode products on the p vectors with the
//            combination fused into the last one; phi_0 from exp(-t A^d).
#include <cstdio>
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstring>
#include <new>
#include <vector>

#include "phiq.h"
#include "phiq_internal.h"

#define PHIQ_HIP(x)                               \
  do {                                            \
    hipError_t e_ = (hipError_t)(x);              \
    if (e_ != hipSuccess) return PHIQ_ERR_HIP;    \
  } while (0)
#define PHIQ_TRY(x)                  \
  do {                               \
    phiq_status s_ = (x);            \
    if (s_ != PHIQ_OK) return s_;    \
  } while (0)

namespace phiq {

constexpr double kThetaMax = 2.0;  // Taylor series is used for ||Z||_inf <= 2
constexpr int kMaxTaylor = 32;
constexpr size_t kAlign = 256;

inline size_t align_up(size_t x) { return (x + kAlign - 1) / kAlign * kAlign; }

struct DevBuf {
  void* p = nullptr;
  size_t cap = 0;
};

struct Staging {
  void* host[3] = {nullptr, nullptr, nullptr};
  size_t cap[3] = {0, 0, 0};
  hipEvent_t ev[3] = {nullptr, nullptr, nullptr};
  bool pending[3] = {false, false, false};
  int next = 0;
};

// Smallest K with nu^{K+1}/(K+1)! / (1 - nu/(K+2)) <= 2^-54 (Taylor remainder
// of exp for ||Z|| <= nu), at least 1.
int taylor_degree(double nu) {
  if (nu <= 0.0) return 1;
  double term = nu;  // nu^{K+1}/(K+1)! for K = 0
  for (int K = 1; K <= kMaxTaylor; ++K) {
    term *= nu / (K + 1);
    const double tail = term / (1.0 - nu / (K + 2));
    if (nu < K + 2 && tail <= std::ldexp(1.0, -54)) return K;
  }
  return kMaxTaylor;
}

double infnorm(const double* A, int n) {
  double best = 0.0;
  for (int i = 0; i < n; ++i) {
    double s = 0.0;
    for (int j = 0; j < n; ++j) s += std::fabs(A[(size_t)i * n + j]);
    best = std::max(best, s);
  }
  return best;
}

phiq_status validate_op(const phiq_kron_op* op) {
  if (!op || op->dim < 1 || op->dim > PHIQ_MAX_DIM) return PHIQ_ERR_INVALID_ARG;
  long double N = 1;
  for (int d = 0; d < op->dim; ++d) {
    if (op->n[d] < 1 || op->n[d] > PHIQ_MAX_N || !op->A[d]) return PHIQ_ERR_INVALID_ARG;
    N *= op->n[d];
  }
  if (N > (long double)(1LL << 36)) return PHIQ_ERR_INVALID_ARG;
  for (int d = 0; d < op->dim; ++d)
    if (N / op->n[d] >= (long double)(1LL << 31)) return PHIQ_ERR_INVALID_ARG;
  for (int d = 0; d < op->dim; ++d) {
    const size_t nn = (size_t)op->n[d] * op->n[d];
    for (size_t i = 0; i < nn; ++i)
      if (!std::isfinite(op->A[d][i])) return PHIQ_ERR_NONFINITE;
  }
  return PHIQ_OK;
}

double sum_infnorms(const phiq_kron_op* op) {
  double s = 0.0;
  for (int d = 0; d < op->dim; ++d) s += infnorm(op->A[d], op->n[d]);
  return s;
}

// Host part of a plan: norm estimate (eq. infnorm_upper_bnd), (l, m) by the
// selector with beta = 1, the 1D scaling sigma_d of each Taylor argument and
// the Taylor degree.  Shared by single plans and batches so both choose the
// same parameters for the same problem.
phiq_status select_params(const phiq_kron_op* op, double t, int p, double tol, const phiq_options& opt,
                          PlanParams* pp, const float* mlp) {
  double norms[PHIQ_MAX_DIM];
  double alpha = 0.0;
  for (int d = 0; d < op->dim; ++d) {
    norms[d] = std::fabs(t) * infnorm(op->A[d], op->n[d]);
    alpha += norms[d];
  }
  if (opt.alpha >= 0) alpha = opt.alpha;
  pp->alpha = alpha;
  pp->log10_bound = 0.0;
  pp->selector = 0;
  int l = 0, nq = -1;
  if (p > 0) {
    double cost = 0.0;
    if (opt.l >= 0) {
      l = opt.l;
      nq = (opt.rule == PHIQ_RULE_GAUSS)
               ? (opt.m > 0 ? opt.m - 1
                            : (alpha <= 1e-12 ? std::max(1, (p + 1) / 2) - 1
                                              : quadnodes(tol, p, std::ldexp(alpha, -l), 1.0, opt.rule)))
               : 4;
    } else {
      setup_quadrature(tol, p, alpha, 1.0, opt.rule, opt.c1, opt.c2, op->dim, &l, &nq, &cost);
      if (opt.selector == PHIQ_SEL_MLP && mlp && opt.rule == PHIQ_RULE_GAUSS && opt.m <= 0 && alpha > 1e-12 &&
          l >= 0 && nq >= 0) {
        int lm = l, nm = nq, used = 0;
        if (mlp_choose(mlp, op, norms, t, p, tol, std::pow(10.0, opt.selector_slack), alpha, l, nq, &lm, &nm,
                       &used)) {
          l = lm;
          nq = nm;
        }
        pp->selector = used;
      }
      if (opt.m > 0 && opt.rule == PHIQ_RULE_GAUSS) nq = opt.m - 1;
    }
    if (l < 0 || nq < 0) return PHIQ_ERR_NOT_CONVERGED;
    pp->log10_bound = (alpha > 1e-12 && nq >= 1)
                          ? log_quaderr(nq, p, std::ldexp(alpha, -l), 1.0, opt.rule) / std::log(10.0)
                          : -INFINITY;
  }
  pp->l = l;
  pp->m = (p > 0 && opt.rule == PHIQ_RULE_GAUSS) ? nq + 1 : 0;
  double nu = 0.0;
  for (int d = 0; d < op->dim; ++d) {
    const double xd = std::ldexp(norms[d], -l);
    int s = 0;
    while (std::ldexp(xd, -s) > kThetaMax) ++s;
    pp->sigma[d] = s;
    nu = std::max(nu, std::ldexp(xd, -s));
  }
  pp->K = taylor_degree(nu);
  return PHIQ_OK;
}

}  // namespace phiq

using namespace phiq;

struct ProfRec {
  int cls;
  hipEvent_t e0, e1;
  double flops, bytes;
};

struct Profiler {
  bool on = false;    // launches are being bracketed
  bool open = false;  // between phiq_profile_start and phiq_profile_stop
  unsigned mask = ~0u;
  std::vector<ProfRec> recs;
  std::vector<hipEvent_t> pool;
  size_t next = 0;
};

static const char* const kProfClass[] = {"ttm_store", "ttm_accum", "ttm_square", "gemm",  "taylor",
                                         "scale",     "node_sum",  "absdiff",    "slice", "ttm_slab"};
enum ProfClass {
  K_TTM_STORE = 0,
  K_TTM_ACCUM,
  K_TTM_SQUARE,
  K_GEMM,
  K_TAYLOR,
  K_SCALE,
  K_NODE_SUM,
  K_ABSDIFF,
  K_SLICE,     // int8 digit slicing of factors and tensors
  K_TTM_SLAB,  // products along axes 2 and 1 in one pass (kernels_slab.hip)
  K_NCLASS
};

// FP64 matrix regions and their lower-precision copies (see TtmArgs::Ea)
struct Twin {
  const double* base;
  size_t count;
  void* a;
  void* b;
};
struct TwinMap {
  std::vector<Twin> t;
  void lookup(const double* E, phiq_precision prec, const void** ea, const void** eb) const {
    *ea = nullptr;
    *eb = nullptr;
    for (const auto& w : t) {
      if (E >= w.base && E < w.base + w.count) {
        const size_t idx = (size_t)(E - w.base);
        if (prec == PHIQ_PREC_FP32) {
          *ea = (const float*)w.a + idx;
        } else {
          *ea = (const uint16_t*)w.a + idx;
          *eb = (const uint16_t*)w.b + idx;
        }
        return;
      }
    }
  }
};
inline size_t twin_bytes(size_t count) { return ((count * 4) + 255) / 256 * 256; }
// precisions whose products read FP32 / bf16 copies of the 1D factors
inline bool twin_prec(phiq_precision p) { return p == PHIQ_PREC_FP32 || p == PHIQ_PREC_BF16X3; }

struct TuneEntry {
  int kind, M, L, nb, cfg;
};

struct phiq_handle_s {
  int device = 0;
  Profiler prof;
  hipStream_t aux = nullptr;      // side stream: scaling chain of the 1D factors, phi_0
  hipStream_t ps = nullptr;       // plan stream of phiq_action: the next call's plan overlaps this execution
  hipEvent_t tr_ready = nullptr;  // a one-call plan's factors are ready
  hipStream_t copy = nullptr;     // upload stream of transient plans
  hipEvent_t tr_fork = nullptr;   // fork/join events of transient plans
  hipEvent_t tr_join = nullptr;
  hipEvent_t tr_fork2 = nullptr;  // phi_0 on the side stream: start / done
  hipEvent_t tr_phi0 = nullptr;
  // transient plans alternate between two buffers so the upload of the next
  // call overlaps the execution of the current one
  DevBuf tr_buf[2];
  // adaptive Clenshaw-Curtis node tables of transient plans, per slot and
  // level (kept like tr_buf, so that a call neither allocates nor frees them)
  std::vector<DevBuf> tr_cc[2];
  hipEvent_t tr_free[2] = {nullptr, nullptr};  // buffer no longer read
  hipEvent_t tr_up[2] = {nullptr, nullptr};    // upload into buffer done
  bool tr_used[2] = {false, false};
  int tr_next = 0;
  // captured device work of phiq_action, keyed by everything the captured
  // launches depend on (pointers, shapes, plan parameters)
  struct GraphEntry {
    std::vector<long long> key;
    hipGraphExec_t exec;
  };
  std::vector<GraphEntry> graphs;
  std::vector<std::vector<long long>> seen;  // keys run once eagerly
  std::vector<TuneEntry> tune;  // fastest tile shape per launch shape (autotuner)
  int force_cfg[5] = {-1, -1, -1, -1, -1};  // phiq_tile_config: one shape for every launch of a kind
  // adaptive Clenshaw-Curtis: the device decisions per level, their pinned
  // host copies and events, and the flag that guards the launches of a
  // speculative level (set only while such a level is enqueued)
  DevBuf cc_ctl;
  CcCtl* cc_ctl_host = nullptr;
  std::vector<hipEvent_t> cc_ev;
  const int* guard = nullptr;
  DevBuf ws;                     // execute workspace (T0, T1, Ya, Yb)
  DevBuf scratch;                // transient plans (phiq_action) and phiq_expm
  std::vector<DevBuf> cc_levels; // node vectors of the adaptive rule, per level
  DevBuf partial;                // CC reduction partials
  DevBuf combo_coef;             // node-sum coefficients of a Clenshaw-Curtis linear combination
  double* partial_host = nullptr;
  DevBuf batch;                  // phiq_action_batched: factors, workspaces, stage tables
  std::vector<float> mlp;        // selector network (phiq_selector_set), empty if none
  Staging stage;
  size_t cap_bytes = 0;
  size_t held() const {
    size_t s = ws.cap + scratch.cap + partial.cap + combo_coef.cap + tr_buf[0].cap + tr_buf[1].cap + batch.cap;
    for (const auto& b : cc_levels) s += b.cap;
    for (int k = 0; k < 2; ++k)
      for (const auto& b : tr_cc[k]) s += b.cap;
    return s;
  }
};

struct phiq_plan_s {
  phiq_handle h = nullptr;
  bool transient = false;
  void* mem = nullptr;
  size_t bytes = 0;
  int D = 0;
  int n[PHIQ_MAX_DIM] = {};
  long long N = 1;
  double t = 0.0;
  int p = 0;
  double tol = 0.0;
  phiq_options opt{};
  int l = 0, m = 0, K = 1;
  int sigma[PHIQ_MAX_DIM] = {};
  int selector = 0;  // phiq_report::selector
  double alpha = 0.0, log10_bound = 0.0;
  // max_i (-A_ii + sum_{j != i} |A_ij|) per axis: ||e^{-cA^d}||_inf <= e^{c mu}
  double mu[PHIQ_MAX_DIM] = {};
  // device pointers (inside mem)
  double* Z[PHIQ_MAX_DIM] = {};      // Z^1..Z^K
  double* Enode[PHIQ_MAX_DIM] = {};  // Gauss: m node slots then phi_0; CC: phi_0 only
  double* Esq[PHIQ_MAX_DIM] = {};    // E^(0)..E^(l-1)
  double* Ephi0[PHIQ_MAX_DIM] = {};
  double* S[2][PHIQ_MAX_DIM] = {};   // ping-pong for the sigma squarings
  double* coef = nullptr;            // p x ldcoef
  int ldcoef = 0;
  char* jobs = nullptr;              // device job tables (per upload)
  size_t jobs_cap = 0;
  TwinMap twins;  // lower-precision copies of the matrices
  // The chain E^(k) = E^(k-1)^2 runs on the handle's side stream while the
  // quadrature runs; the executing stream waits on `join` before it needs
  // E^(k) (squaring) or E^(l) (phi_0).
  hipEvent_t fork = nullptr, join = nullptr;
  hipEvent_t fork2 = nullptr, phi0 = nullptr;  // phi_0 on the side stream
  bool own_events = false, has_join = false;
  bool single_stream = false;  // everything on the caller's stream (graph capture)
  int tr_slot = -1;  // transient buffer used (phiq_action)
  void* ej = nullptr;  // the plan's device job groups (ExpmJobs), enqueued by plan_enqueue
  void (*ej_free)(void*) = nullptr;
  // adaptive Clenshaw-Curtis: per level, node exponentials [axis][count]
  // (owned by the plan, or by the handle's transient slot when cc_pooled)
  std::vector<DevBuf> cc_E;
  std::vector<int> cc_count;
  bool cc_pooled = false;
  ~phiq_plan_s() {
    if (ej && ej_free) ej_free(ej);
    if (own_events) {
      if (fork) (void)hipEventDestroy(fork);
      if (join) (void)hipEventDestroy(join);
      if (fork2) (void)hipEventDestroy(fork2);
      if (phi0) (void)hipEventDestroy(phi0);
    }
    if (!cc_pooled)
      for (auto& b : cc_E)
        if (b.p) (void)hipFree(b.p);
    if (!transient && mem) (void)hipFree(mem);
  }
};

namespace {

struct DeviceGuard {
  int prev = -1;
  explicit DeviceGuard(int dev) {
    if (hipGetDevice(&prev) != hipSuccess) prev = -1;
    if (prev != dev) (void)hipSetDevice(dev);
  }
  ~DeviceGuard() {
    int cur = -1;
    if (prev >= 0 && hipGetDevice(&cur) == hipSuccess && cur != prev) (void)hipSetDevice(prev);
  }
};

hipEvent_t prof_event(phiq_handle h) {
  Profiler& pr = h->prof;
  if (pr.next < pr.pool.size()) return pr.pool[pr.next++];
  hipEvent_t e = nullptr;
  if (hipEventCreate(&e) != hipSuccess) return nullptr;
  pr.pool.push_back(e);
  pr.next = pr.pool.size();
  return e;
}

// Launch through f() (exactly one kernel); when this class is profiled the
// kernel's dispatch carries a start and a stop event.
template <class F>
phiq_status prof_launch(phiq_handle h, hipStream_t st, int cls, double flops, double bytes, F&& f) {
  hipEvent_t e0 = nullptr, e1 = nullptr;
  const bool rec = h->prof.on && ((h->prof.mask >> cls) & 1u);
  if (rec) {
    e0 = prof_event(h);
    e1 = prof_event(h);
    if (e0 && e1) {
      g_launch_events[0] = e0;
      g_launch_events[1] = e1;
    }
  }
  (void)st;
  const int err = f();
  g_launch_events[0] = g_launch_events[1] = nullptr;
  if (err != hipSuccess) return PHIQ_ERR_HIP;
  if (rec && e0 && e1) h->prof.recs.push_back({cls, e0, e1, flops, bytes});
  return PHIQ_OK;
}

// Algorithmic work of a batched mode product (see TtmArgs).
void ttm_work(const TtmArgs& a, int cls, double* flops, double* bytes) {
  const double N = (double)a.L * a.K;
  *flops = 2.0 * a.M * a.K * (double)a.L * a.nbatch;
  const double xin = (a.xs == 0 ? 1.0 : (double)a.nbatch) * N;
  double out = (double)a.nbatch * a.M * a.L;
  double extra = 0.0;
  if (cls == K_TTM_ACCUM) out = (double)a.np * a.M * a.L;
  if (cls == K_TTM_SQUARE) extra = (double)(a.nbatch + a.order0) * a.M * a.L;  // the y_j read once
  if (a.yacc) extra += out;  // the previous output read back
  const double xb = a.x_f32 ? 4.0 : 8.0;
  const double ob = (a.o_f32 && cls == K_TTM_STORE) ? 4.0 : 8.0;
  *bytes = xb * xin + ob * out + 8.0 * (extra + (double)a.nbatch * a.M * a.K * (a.es == 0 ? 0.0 : 1.0));
}

int tuned_cfg(phiq_handle h, int kind, const TtmArgs& a) {
  const int nb = (kind == 1) ? 1 : a.nbatch;
  for (const auto& e : h->tune)
    if (e.kind == kind && e.M == a.M && e.L == a.L && e.nb == nb) return e.cfg;
  return -1;
}

// Without a tuned entry: the shapes the autotuner picks at n = 128 (stores:
// 64 x 128 eight-wave tiles when they fill the GPU, 64 x 64 tiles with
// 32-deep chunks when they would not; node sums: 64 x 64, eight waves;
// squaring: all orders per block, eight waves), else the kernels' defaults.
int fallback_cfg(int kind, const TtmArgs& a) {
  if (kind == 0 && a.M >= 128) {
    const long long tiles = (long long)((a.M + 63) / 64) * ((a.L + 127) / 128) * a.nbatch;
    return tiles < 768 ? 6 : 11;
  }
  if (kind == 1 && a.M >= 128) return 6;  // node sum: 64 x 64 tiles, eight waves
  if (kind == 2 && a.M >= 128 && a.nbatch <= 4 && a.es == 0) return 11;
  return -1;
}

int launch_kind(int kind, const TtmArgs& a, phiq_precision prec, hipStream_t st, int cfg) {
  if (kind == 1) return launch_ttm_accum(a, prec, st, cfg);
  if (kind == 2) return launch_ttm_square(a, prec, st, cfg);
  return launch_ttm_store(a, prec, st, cfg);
}

int kind_of(int cls) { return cls == K_TTM_ACCUM ? 1 : (cls == K_TTM_SQUARE ? 2 : 0); }

phiq_status L_ttm(phiq_handle h, int cls, const TtmArgs& a0, phiq_precision prec, hipStream_t st,
                  const TwinMap* tw = nullptr) {
  double fl, by;
  TtmArgs a = a0;
  a.stop = h->guard;
  if (prec != PHIQ_PREC_FP64) {
    if (!tw) return PHIQ_ERR_INVALID_ARG;
    tw->lookup(a.E, prec, &a.Ea, &a.Eb);
    if (!a.Ea) return PHIQ_ERR_INVALID_ARG;
  }
  double f = 1.0;
  for (int k = 0; k <= PHIQ_MAX_P; ++k) {
    a.ifact[k] = 1.0 / f;
    f *= (k + 1);
  }
  ttm_work(a, cls, &fl, &by);
  const int kind = kind_of(cls);
  // split bf16: kinds 3 / 4 force the resident-factor shapes of the plain
  // and the squaring products (0 = the general tile kernel)
  int cfg = (prec == PHIQ_PREC_BF16X3 && kind != 1) ? h->force_cfg[kind == 0 ? 3 : 4]
            : (prec != PHIQ_PREC_FP64) ? -1
                                       : (h->force_cfg[kind] >= 0 ? h->force_cfg[kind] : tuned_cfg(h, kind, a));
  if (prec == PHIQ_PREC_FP64 && cfg < 0) cfg = fallback_cfg(kind, a);
  return prof_launch(h, st, cls, fl, by, [&] { return launch_kind(kind, a, prec, st, cfg); });
}

phiq_status L_gemm(phiq_handle h, const GemmJob* jobs, int njobs, int nm, hipStream_t st) {
  const double n = nm;
  return prof_launch(h, st, K_GEMM, 2.0 * n * n * n * njobs, 24.0 * n * n * njobs,
                     [&] { return launch_gemm_jobs(jobs, njobs, nm, st); });
}

phiq_status L_taylor(phiq_handle h, const TaylorJob* jobs, int njobs, int nm, int K, hipStream_t st) {
  const double n = nm;
  return prof_launch(h, st, K_TAYLOR, 2.0 * K * n * n * njobs, 8.0 * (K + 1) * n * n * njobs,
                     [&] { return launch_taylor_jobs(jobs, njobs, nm, st); });
}

phiq_status L_scale(phiq_handle h, const ScaleJob* jobs, int njobs, int nm, hipStream_t st) {
  const double n = nm;
  return prof_launch(h, st, K_SCALE, n * n * njobs, 16.0 * n * n * njobs,
                     [&] { return launch_scale_jobs(jobs, njobs, nm, st); });
}

phiq_status ensure(phiq_handle h, DevBuf& b, size_t bytes) {
  if (bytes <= b.cap) return PHIQ_OK;
  const size_t want = align_up(bytes + bytes / 8);
  if (h->cap_bytes && h->held() - b.cap + want > h->cap_bytes) {
    if (h->held() - b.cap + bytes > h->cap_bytes) return PHIQ_ERR_OOM;
  }
  size_t get = want;
  if (h->cap_bytes && h->held() - b.cap + get > h->cap_bytes) get = align_up(bytes);
  if (b.p) {
    PHIQ_HIP(hipDeviceSynchronize());
    PHIQ_HIP(hipFree(b.p));
    b.p = nullptr;
    b.cap = 0;
  }
  if (hipMalloc(&b.p, get) != hipSuccess) {
    b.p = nullptr;
    (void)hipGetLastError();
    return PHIQ_ERR_OOM;
  }
  b.cap = get;
  return PHIQ_OK;
}

// Pinned staging buffer for one host->device copy; waits if the slot's
// previous copy has not run yet.
phiq_status stage_acquire(phiq_handle h, size_t bytes, int* slot, void** host) {
  Staging& s = h->stage;
  const int k = s.next;
  s.next = (s.next + 1) % 3;
  if (s.pending[k]) {
    PHIQ_HIP(hipEventSynchronize(s.ev[k]));
    s.pending[k] = false;
  }
  if (s.cap[k] < bytes) {
    if (s.host[k]) PHIQ_HIP(hipHostFree(s.host[k]));
    s.host[k] = nullptr;
    s.cap[k] = 0;
    const size_t want = align_up(std::max(bytes, (size_t)1 << 16));
    if (hipHostMalloc(&s.host[k], want, hipHostMallocDefault) != hipSuccess) {
      s.host[k] = nullptr;
      return PHIQ_ERR_OOM;
    }
    s.cap[k] = want;
  }
  if (!s.ev[k]) PHIQ_HIP(hipEventCreateWithFlags(&s.ev[k], hipEventDisableTiming));
  *slot = k;
  *host = s.host[k];
  return PHIQ_OK;
}

phiq_status stage_copy(phiq_handle h, int slot, void* dst, size_t bytes, hipStream_t st) {
  PHIQ_HIP(hipMemcpyAsync(dst, h->stage.host[slot], bytes, hipMemcpyHostToDevice, st));
  PHIQ_HIP(hipEventRecord(h->stage.ev[slot], st));
  h->stage.pending[slot] = true;
  return PHIQ_OK;
}

// Staged upload through a kernel that reads the pinned host buffer.
phiq_status stage_fetch(phiq_handle h, int slot, void* dst, size_t bytes, hipStream_t st) {
  PHIQ_HIP(launch_fetch(dst, h->stage.host[slot], bytes, st));
  PHIQ_HIP(hipEventRecord(h->stage.ev[slot], st));
  h->stage.pending[slot] = true;
  return PHIQ_OK;
}

// Simple bump layout of one device allocation.
struct Layout {
  size_t off = 0;
  size_t take(size_t bytes) {
    const size_t o = off;
    off = align_up(off + bytes);
    return o;
  }
};

// Host-side builder of a job blob: jobs are appended and later uploaded as
// one copy; each group remembers its offset and count.
struct JobBlob {
  std::vector<char> bytes;
  template <class T>
  size_t add(const std::vector<T>& v) {
    const size_t o = align_up(bytes.size());
    bytes.resize(o + v.size() * sizeof(T));
    if (!v.empty()) std::memcpy(bytes.data() + o, v.data(), v.size() * sizeof(T));
    bytes.resize(align_up(bytes.size()));
    return o;
  }
};

struct ExpmJobs {
  // offsets into the blob and counts
  size_t scale_off = 0;
  int scale_n = 0;
  std::vector<std::pair<size_t, int>> power_rounds;
  size_t taylor_off = 0;
  int taylor_n = 0;
  std::vector<std::pair<size_t, int>> sigma_rounds;
  std::vector<std::pair<size_t, int>> square_chain;
};

// Target of one Taylor evaluation: axis d, coefficient c, final slot.
struct ExpTarget {
  int d;
  double c;
  double* dst;
  int sidx;  // slot index in the sigma ping-pong buffers
};

// Jobs: powers of Z_d (already scaled in place), Taylor series for every
// target, and sigma_d squarings through the ping-pong slots.
void build_taylor_and_sigma(const phiq_plan_s* P, const std::vector<ExpTarget>& tg, JobBlob& blob,
                            ExpmJobs& ej) {
  std::vector<TaylorJob> tj;
  int smax = 0;
  for (int d = 0; d < P->D; ++d) {
    const int n = P->n[d];
    TaylorJob j{};
    for (const auto& t : tg) {
      if (t.d != d) continue;
      if (j.nt == kTaylorTargets) {
        tj.push_back(j);
        j = TaylorJob{};
      }
      j.Zpow = P->Z[d];
      j.n = n;
      j.K = P->K;
      j.c[j.nt] = t.c;
      j.dst[j.nt] = P->sigma[d] > 0 ? P->S[0][d] + (size_t)t.sidx * n * n : t.dst;
      ++j.nt;
      smax = std::max(smax, P->sigma[d]);
    }
    if (j.nt > 0) tj.push_back(j);
  }
  ej.taylor_off = blob.add(tj);
  ej.taylor_n = (int)tj.size();
  for (int r = 1; r <= smax; ++r) {
    std::vector<GemmJob> gj;
    for (const auto& t : tg) {
      const int d = t.d, n = P->n[d];
      if (P->sigma[d] < r) continue;
      const size_t off = (size_t)t.sidx * n * n;
      GemmJob g{};
      const double* src = P->S[(r - 1) % 2][d] + off;
      g.A = src;
      g.B = src;
      g.C = (r == P->sigma[d]) ? t.dst : P->S[r % 2][d] + off;
      g.n = n;
      gj.push_back(g);
    }
    ej.sigma_rounds.push_back({blob.add(gj), (int)gj.size()});
  }
}

void build_powers(const phiq_plan_s* P, JobBlob& blob, ExpmJobs& ej) {
  for (int pw = 1; pw < P->K; pw *= 2) {
    std::vector<GemmJob> gj;
    for (int d = 0; d < P->D; ++d) {
      const size_t nn = (size_t)P->n[d] * P->n[d];
      for (int j = 1; j <= pw && j + pw <= P->K; ++j) {
        GemmJob g{};
        g.A = P->Z[d] + (size_t)(j - 1) * nn;
        g.B = P->Z[d] + (size_t)(pw - 1) * nn;
        g.C = P->Z[d] + (size_t)(j + pw - 1) * nn;
        g.n = P->n[d];
        gj.push_back(g);
      }
    }
    ej.power_rounds.push_back({blob.add(gj), (int)gj.size()});
  }
}

int nmax_of(const phiq_plan_s* P) {
  int nm = 1;
  for (int d = 0; d < P->D; ++d) nm = std::max(nm, P->n[d]);
  return nm;
}

phiq_status run_taylor_sigma(const phiq_plan_s* P, const char* jobs_dev, const ExpmJobs& ej, hipStream_t st) {
  const int nm = nmax_of(P);
  PHIQ_TRY(L_taylor(P->h, (const TaylorJob*)(jobs_dev + ej.taylor_off), ej.taylor_n, nm, P->K, st));
  for (const auto& r : ej.sigma_rounds) PHIQ_TRY(L_gemm(P->h, (const GemmJob*)(jobs_dev + r.first), r.second, nm, st));
  return PHIQ_OK;
}

// Convert count FP64 elements starting at E (inside a twin region) to the
// plan's lower precision.
phiq_status convert_range(const phiq_plan_s* P, const double* E, size_t count, hipStream_t st) {
  for (const auto& w : P->twins.t) {
    if (E >= w.base && E + count <= w.base + w.count) {
      const size_t idx = (size_t)(E - w.base);
      if (P->opt.precision == PHIQ_PREC_FP32) {
        PHIQ_HIP(launch_convert(E, (long long)count, P->opt.precision, (float*)w.a + idx, nullptr, st));
      } else {
        PHIQ_HIP(launch_convert(E, (long long)count, P->opt.precision, (uint16_t*)w.a + idx, (uint16_t*)w.b + idx,
                                st));
      }
      return PHIQ_OK;
    }
  }
  return PHIQ_ERR_INVALID_ARG;
}

phiq_status wait_join(const phiq_plan_s* P, hipStream_t st) {
  if (P->has_join) PHIQ_HIP(hipStreamWaitEvent(st, P->join, 0));
  return PHIQ_OK;
}

// Device work of a plan: the 1D exponentials (all on st, except the scaling
// chain E^(k) = E^(k-1)^2, which forks to the side stream and is joined by
// the executing stream before the squaring and phi_0).  Enqueue only:
// usable under stream capture.
phiq_status plan_enqueue(phiq_plan P, hipStream_t st) {
  phiq_handle h = P->h;
  const ExpmJobs& ej = *(const ExpmJobs*)P->ej;
  const bool lp = twin_prec(P->opt.precision);
  const int l = P->l;
  const int nm = nmax_of(P);
  bool ok = L_scale(h, (const ScaleJob*)(P->jobs + ej.scale_off), ej.scale_n, nm, st) == PHIQ_OK;
  for (const auto& r : ej.power_rounds)
    ok = ok && L_gemm(h, (const GemmJob*)(P->jobs + r.first), r.second, nm, st) == PHIQ_OK;
  ok = ok && run_taylor_sigma(P, P->jobs, ej, st) == PHIQ_OK;
  if (lp)  // node factors (and E^(0) = the phi_0 factor when l = 0)
    for (int d = 0; d < P->D && ok; ++d) {
      const size_t nn = (size_t)P->n[d] * P->n[d];
      ok = convert_range(P, P->Enode[d], nn * P->m, st) == PHIQ_OK;
      if (ok && l == 0) ok = convert_range(P, P->Ephi0[d], nn, st) == PHIQ_OK;
    }
  if (ok && l > 0) {
    hipStream_t cs = P->single_stream ? st : h->aux;
    if (!P->single_stream)
      ok = hipEventRecord(P->fork, st) == hipSuccess && hipStreamWaitEvent(h->aux, P->fork, 0) == hipSuccess;
    for (const auto& r : ej.square_chain)
      ok = ok && L_gemm(h, (const GemmJob*)(P->jobs + r.first), r.second, nm, cs) == PHIQ_OK;
    if (lp)
      for (int d = 0; d < P->D && ok; ++d) {
        const size_t nn = (size_t)P->n[d] * P->n[d];
        ok = convert_range(P, P->Esq[d], nn * l, cs) == PHIQ_OK && convert_range(P, P->Ephi0[d], nn, cs) == PHIQ_OK;
      }
    if (!P->single_stream) {
      ok = ok && hipEventRecord(P->join, h->aux) == hipSuccess;
      P->has_join = ok;
    }
  }
  return ok ? PHIQ_OK : PHIQ_ERR_HIP;
}

// ---------------------------------------------------------------------------
// plan creation
// ---------------------------------------------------------------------------
phiq_status plan_enqueue(phiq_plan P, hipStream_t st);

phiq_status plan_build(phiq_handle h, const phiq_kron_op* op, double t, int p, double tol, const phiq_options* uopt,
                       bool transient, phiq_plan* out, phiq_report* rep, hipStream_t st, bool defer_device = false) {
  if (!h || !out) return PHIQ_ERR_INVALID_ARG;
  PHIQ_TRY(validate_op(op));
  if (!std::isfinite(t) || !std::isfinite(tol)) return PHIQ_ERR_NONFINITE;
  if (p < 0 || p > PHIQ_MAX_P || !(tol > 0)) return PHIQ_ERR_INVALID_ARG;
  phiq_options opt;
  phiq_options_default(&opt);
  if (uopt) opt = *uopt;
  if (opt.rule != PHIQ_RULE_GAUSS && opt.rule != PHIQ_RULE_CC) return PHIQ_ERR_INVALID_ARG;
  if (opt.precision != PHIQ_PREC_FP64 && opt.precision != PHIQ_PREC_FP32 && opt.precision != PHIQ_PREC_BF16X3 &&
      opt.precision != PHIQ_PREC_INT8)
    return PHIQ_ERR_INVALID_ARG;
  if (opt.precision == PHIQ_PREC_INT8) {
    if (opt.rule != PHIQ_RULE_GAUSS || op->dim < 2) return PHIQ_ERR_UNSUPPORTED;
    for (int d = 0; d < op->dim; ++d)
      if (op->n[d] % 32 != 0 || op->n[d] > 128) return PHIQ_ERR_UNSUPPORTED;
  }
  // a tolerance below the lower-precision products' rounding floor cannot be
  // met; refused unless the caller accepts the floor
  if (tol < precision_floor(opt.precision) && !opt.accept_floor) return PHIQ_ERR_UNSUPPORTED;
  if (!std::isfinite(opt.c1) || !std::isfinite(opt.c2) || !std::isfinite(opt.alpha)) return PHIQ_ERR_NONFINITE;
  if (opt.c1 < 0 || opt.c2 < 0 || opt.l < -1 || opt.l > 60 || opt.m < -1 || opt.m == 0 || opt.m > 4096 ||
      opt.cc_max_doublings < 1 || opt.cc_max_doublings > 10 || !(opt.selector_slack >= 0.0) ||
      opt.selector_slack > 12.0)
    return PHIQ_ERR_INVALID_ARG;

  PlanParams pp;
  PHIQ_TRY(select_params(op, t, p, tol, opt, &pp, h->mlp.empty() ? nullptr : h->mlp.data()));
  phiq_plan P = new (std::nothrow) phiq_plan_s;
  if (!P) return PHIQ_ERR_OOM;
  P->h = h;
  P->transient = transient;
  P->D = op->dim;
  for (int d = 0; d < P->D; ++d) {
    P->n[d] = op->n[d];
    P->N *= op->n[d];
    P->sigma[d] = pp.sigma[d];
    const double* A = op->A[d];
    const int nd = op->n[d];
    double mu = -INFINITY;
    for (int i = 0; i < nd; ++i) {
      double r = -A[(size_t)i * nd + i];
      for (int j = 0; j < nd; ++j)
        if (j != i) r += std::fabs(A[(size_t)i * nd + j]);
      mu = std::max(mu, r);
    }
    P->mu[d] = mu;
  }
  P->t = t;
  P->p = p;
  P->tol = tol;
  P->opt = opt;
  P->alpha = pp.alpha;
  P->log10_bound = pp.log10_bound;
  P->l = pp.l;
  P->m = pp.m;
  P->K = pp.K;
  P->selector = pp.selector;
  const int l = P->l;

  // a3: the rule (Gauss); CC nodes are produced level by level at execute time
  std::vector<double> theta, w;
  if (P->m > 0) {
    theta.resize(P->m);
    w.resize(P->m);
    gauss_legendre(P->m, theta.data(), w.data());
  }
  const int ncoefcols = (opt.rule == PHIQ_RULE_GAUSS) ? P->m : 7 * (1 << opt.cc_max_doublings) + 1;
  P->ldcoef = std::max(1, ncoefcols);

  // device layout
  // The upload region [A^0 .. A^{D-1} | coef | jobs] comes first so that
  // one host->device copy fills it.
  Layout L;
  size_t offA[PHIQ_MAX_DIM], offZ[PHIQ_MAX_DIM], offE[PHIQ_MAX_DIM], offSq[PHIQ_MAX_DIM], offS0[PHIQ_MAX_DIM],
      offS1[PHIQ_MAX_DIM], offPhi0[PHIQ_MAX_DIM];
  for (int d = 0; d < P->D; ++d) offA[d] = L.take((size_t)P->n[d] * P->n[d] * sizeof(double));
  const size_t coef_bytes = sizeof(double) * (size_t)std::max(1, p) * P->ldcoef;
  const size_t offCoef = L.take(coef_bytes);
  const size_t jobs_cap = 1 << 20;
  const size_t offJobs = L.take(jobs_cap);
  const int nslots = P->m + 1;  // Taylor targets: nodes + E^(0)
  for (int d = 0; d < P->D; ++d) {
    const size_t nn = (size_t)P->n[d] * P->n[d] * sizeof(double);
    offZ[d] = L.take(nn * P->K);
    offE[d] = L.take(nn * (P->m + 1));
    offSq[d] = L.take(nn * std::max(1, l));
    offPhi0[d] = (opt.rule == PHIQ_RULE_GAUSS) ? offE[d] + nn * P->m : L.take(nn);
    const int cc_slots = (opt.rule == PHIQ_RULE_CC) ? 3 * (1 << opt.cc_max_doublings) + 1 : nslots;
    const int ss = std::max(nslots, cc_slots);
    offS0[d] = P->sigma[d] > 0 ? L.take(nn * ss) : 0;
    offS1[d] = P->sigma[d] > 1 ? L.take(nn * ss) : 0;
  }
  const size_t nconv = L.off / sizeof(double);  // every matrix of the plan lies below here
  const bool lp = twin_prec(opt.precision);
  const size_t offTwin = lp ? L.take(twin_bytes(nconv)) : 0;
  P->bytes = L.off;
  if (transient) {
    const int k = h->tr_next;
    h->tr_next ^= 1;
    // the call before last used this buffer: its execution must be done
    // before the upload (on st) overwrites it
    if (h->tr_used[k] && h->tr_free[k] && hipStreamWaitEvent(st, h->tr_free[k], 0) != hipSuccess) {
      delete P;
      return PHIQ_ERR_HIP;
    }
    phiq_status s = ensure(h, h->tr_buf[k], P->bytes);
    if (s != PHIQ_OK) {
      delete P;
      return s;
    }
    P->mem = h->tr_buf[k].p;
    P->tr_slot = k;
  } else {
    if (h->cap_bytes && h->held() + P->bytes > h->cap_bytes) {
      delete P;
      return PHIQ_ERR_OOM;
    }
    if (hipMalloc(&P->mem, P->bytes) != hipSuccess) {
      P->mem = nullptr;
      (void)hipGetLastError();
      delete P;
      return PHIQ_ERR_OOM;
    }
  }
  char* base = (char*)P->mem;
  for (int d = 0; d < P->D; ++d) {
    P->Z[d] = (double*)(base + offZ[d]);
    P->Enode[d] = (double*)(base + offE[d]);
    P->Esq[d] = (double*)(base + offSq[d]);
    P->Ephi0[d] = (double*)(base + offPhi0[d]);
    P->S[0][d] = P->sigma[d] > 0 ? (double*)(base + offS0[d]) : nullptr;
    P->S[1][d] = P->sigma[d] > 1 ? (double*)(base + offS1[d]) : nullptr;
  }
  P->coef = (double*)(base + offCoef);
  P->jobs = base + offJobs;
  P->jobs_cap = jobs_cap;
  if (lp) {
    char* tb = base + offTwin;
    P->twins.t.push_back({(const double*)base, nconv, tb, tb + nconv * 2});
  }

  // ---- host blob: A^d, coefficients, job tables ----
  JobBlob blob;
  ExpmJobs ej;
  // scale jobs: Z_d^1 = (-t 2^{-l-sigma_d}) A^d (A^d uploaded into its slot)
  std::vector<ScaleJob> sj;
  for (int d = 0; d < P->D; ++d) {
    ScaleJob s{};
    s.src = (const double*)(base + offA[d]);
    s.dst = P->Z[d];
    s.s = -t * std::ldexp(1.0, -l - P->sigma[d]);
    s.n = P->n[d];
    sj.push_back(s);
  }
  ej.scale_off = blob.add(sj);
  ej.scale_n = (int)sj.size();
  build_powers(P, blob, ej);
  // Taylor targets: Gauss nodes (c = 1 - theta_q) and E^(0) (c = 1)
  std::vector<ExpTarget> tg;
  for (int d = 0; d < P->D; ++d) {
    const size_t nn = (size_t)P->n[d] * P->n[d];
    for (int q = 0; q < P->m; ++q) tg.push_back({d, 1.0 - theta[q], P->Enode[d] + q * nn, q});
    tg.push_back({d, 1.0, l > 0 ? P->Esq[d] : P->Ephi0[d], P->m});
  }
  build_taylor_and_sigma(P, tg, blob, ej);
  // E^(k) = E^(k-1)^2, k = 1..l (E^(l) is the phi_0 factor)
  for (int k = 1; k <= l; ++k) {
    std::vector<GemmJob> gj;
    for (int d = 0; d < P->D; ++d) {
      const size_t nn = (size_t)P->n[d] * P->n[d];
      GemmJob g{};
      g.A = P->Esq[d] + (k - 1) * nn;
      g.B = g.A;
      g.C = (k < l) ? P->Esq[d] + k * nn : P->Ephi0[d];
      g.n = P->n[d];
      gj.push_back(g);
    }
    ej.square_chain.push_back({blob.add(gj), (int)gj.size()});
  }
  if (blob.bytes.size() > jobs_cap) {
    phiq_plan_destroy(P);
    return PHIQ_ERR_UNSUPPORTED;
  }
  // one copy: [A^d ...][coef][jobs] mirrored in the staging buffer
  const size_t total = offJobs + blob.bytes.size();
  int slot;
  void* hostp;
  phiq_status s = stage_acquire(h, total, &slot, &hostp);
  if (s != PHIQ_OK) {
    phiq_plan_destroy(P);
    return s;
  }
  char* hp = (char*)hostp;
  for (int d = 0; d < P->D; ++d)
    std::memcpy(hp + offA[d], op->A[d], (size_t)P->n[d] * P->n[d] * sizeof(double));
  double* hc = (double*)(hp + offCoef);
  std::fill(hc, hc + (size_t)std::max(1, p) * P->ldcoef, 0.0);
  if (opt.rule == PHIQ_RULE_GAUSS) {
    for (int j = 0; j < p; ++j) {
      double fact = 1.0;
      for (int k = 2; k <= j; ++k) fact *= k;
      for (int q = 0; q < P->m; ++q) hc[(size_t)j * P->ldcoef + q] = w[q] * std::pow(theta[q], j) / fact;
    }
  }
  std::memcpy(hp + offJobs, blob.bytes.data(), blob.bytes.size());
  // upload: a copy kernel on the caller's stream reads the pinned staging
  // buffer directly (no DMA engine hop, so no cross-engine wait)
  if (stage_fetch(h, slot, base, total, st) != PHIQ_OK) {
    phiq_plan_destroy(P);
    return PHIQ_ERR_HIP;
  }
  // events and the side stream are host set-up (never inside a capture)
  bool ok = true;
  if (l > 0) {
    if (!h->aux) ok = hipStreamCreateWithFlags(&h->aux, hipStreamNonBlocking) == hipSuccess;
    if (ok && transient) {
      hipEvent_t* evs[4] = {&h->tr_fork, &h->tr_join, &h->tr_fork2, &h->tr_phi0};
      for (auto e : evs)
        if (ok && !*e) ok = hipEventCreateWithFlags(e, hipEventDisableTiming) == hipSuccess;
      P->fork = h->tr_fork;
      P->join = h->tr_join;
      P->fork2 = h->tr_fork2;
      P->phi0 = h->tr_phi0;
    } else if (ok) {
      ok = hipEventCreateWithFlags(&P->fork, hipEventDisableTiming) == hipSuccess &&
           hipEventCreateWithFlags(&P->join, hipEventDisableTiming) == hipSuccess &&
           hipEventCreateWithFlags(&P->fork2, hipEventDisableTiming) == hipSuccess &&
           hipEventCreateWithFlags(&P->phi0, hipEventDisableTiming) == hipSuccess;
      P->own_events = true;
    }
  }
  P->ej = new (std::nothrow) ExpmJobs(ej);
  P->ej_free = [](void* q) { delete (ExpmJobs*)q; };
  if (!ok || !P->ej) {
    phiq_plan_destroy(P);
    return PHIQ_ERR_HIP;
  }
  if (!defer_device) {
    const phiq_status sd = plan_enqueue(P, st);
    if (sd != PHIQ_OK) {
      phiq_plan_destroy(P);
      return sd;
    }
  }
  if (rep) {
    std::memset(rep, 0, sizeof(*rep));
    rep->l = P->l;
    rep->m = P->m;
    rep->alpha = P->alpha;
    rep->log10_bound = P->log10_bound;
    rep->selector = P->selector;
    rep->workspace_bytes = h->held();
    rep->precision_floor = precision_floor(P->opt.precision);
    rep->tol_met = P->tol >= rep->precision_floor;
  }
  *out = P;
  return PHIQ_OK;
}

// ---------------------------------------------------------------------------
// execution helpers
// ---------------------------------------------------------------------------
struct Front {
  const void* X;
  long long xs;
  int f32;  // X holds FP32 values
  int nn;   // X is in the natural layout (after the slab product)
};

inline bool lowp(const phiq_plan_s* P) { return twin_prec(P->opt.precision); }
inline size_t tensor_elem(const phiq_plan_s* P) { return lowp(P) ? sizeof(float) : sizeof(double); }
inline const void* elem_offset(const void* X, long long elems, int f32) {
  return (const char*)X + elems * (f32 ? (long long)sizeof(float) : (long long)sizeof(double));
}

// Mode products over axes D-1..1 for nb batches (rotated layout); returns the
// input of the final product over axis 0.  X is FP64; the intermediates T0
// and T1 are FP32 when a lower precision is selected.
phiq_status chain_front(const phiq_plan_s* P, const double* X, long long xs, double* const* Ebase, long long const* es,
                        int nb, void* T0, void* T1, hipStream_t st, Front* f, bool beside = false) {
  // 1: single-vector chains only (with a batch the per-axis kernels keep more
  // waves per CU busy and were faster at n = 128), and not beside other work
  // on a side stream, where a block that takes a whole CU's LDS waits for a
  // free CU
  const int sp = P->opt.slab_products;
  if (P->D == 3 && P->n[1] == kSlabN && P->n[2] == kSlabN && P->opt.precision == PHIQ_PREC_FP64 && !P->h->guard &&
      (sp == 2 || (sp == 1 && nb == 1 && !beside))) {
    SlabArgs s{};
    s.X = X;
    s.xs = xs;
    s.E1 = Ebase[1];
    s.es1 = es[1];
    s.E2 = Ebase[2];
    s.es2 = es[2];
    s.O = (double*)T0;
    s.os = P->N;
    s.n0 = P->n[0];
    s.nbatch = nb;
    if (slab2_supported(s)) {
      const double slabs = (double)s.n0 * nb;
      const double S3 = (double)kSlabN * kSlabN * kSlabN;
      // two 128-deep contractions per element; X read (once when shared), O written, the factors read
      const double bytes = 8.0 * ((xs == 0 ? (double)P->N : slabs * kSlabN * kSlabN) + slabs * kSlabN * kSlabN +
                                  (double)kSlabN * kSlabN * ((es[1] ? nb : 1) + (es[2] ? nb : 1)));
      PHIQ_TRY(prof_launch(P->h, st, K_TTM_SLAB, 4.0 * S3 * slabs, bytes, [&] { return launch_slab2(s, st); }));
      f->X = T0;
      f->xs = P->N;
      f->f32 = 0;
      f->nn = 1;
      return PHIQ_OK;
    }
  }
  const void* cur = X;
  long long cxs = xs;
  int cur_f32 = 0;
  for (int s = 0; s + 1 < P->D; ++s) {
    const int d = P->D - 1 - s;
    TtmArgs a{};
    a.E = Ebase[d];
    a.es = es[d];
    a.X = cur;
    a.xs = cxs;
    a.x_f32 = cur_f32;
    a.O = (s % 2 == 0) ? T0 : T1;
    a.os = P->N;
    a.o_f32 = lowp(P) ? 1 : 0;
    a.M = a.K = P->n[d];
    a.L = (int)(P->N / P->n[d]);
    a.nbatch = nb;
    PHIQ_TRY(L_ttm(P->h, K_TTM_STORE, a, P->opt.precision, st, &P->twins));
    cur = a.O;
    cxs = P->N;
    cur_f32 = a.o_f32;
  }
  f->X = cur;
  f->xs = cxs;
  f->f32 = cur_f32;
  f->nn = 0;
  return PHIQ_OK;
}

TtmArgs final_args(const phiq_plan_s* P, const double* E, long long es, const Front& f, int nb) {
  TtmArgs a{};
  a.E = E;
  a.es = es;
  a.X = f.X;
  a.xs = f.xs;
  a.x_f32 = f.f32;
  a.nn = f.nn;
  a.o_f32 = 0;
  a.M = a.K = P->n[0];
  a.L = (int)(P->N / P->n[0]);
  a.nbatch = nb;
  return a;
}

phiq_status phi0_chain(const phiq_plan_s* P, const double* v, double* out0, void* T0, void* T1, hipStream_t st,
                       bool side = false) {
  if (!side) PHIQ_TRY(wait_join(P, st));
  double* E[PHIQ_MAX_DIM];
  long long es[PHIQ_MAX_DIM];
  for (int d = 0; d < P->D; ++d) {
    E[d] = P->Ephi0[d];
    es[d] = 0;
  }
  Front f;
  PHIQ_TRY(chain_front(P, v, 0, E, es, 1, T0, T1, st, &f, side));
  TtmArgs a = final_args(P, P->Ephi0[0], 0, f, 1);
  a.O = out0;
  a.os = 0;
  PHIQ_TRY(L_ttm(P->h, K_TTM_STORE, a, P->opt.precision, st, &P->twins));
  return PHIQ_OK;
}

// phi_0 on the side stream, after the scaling chain there (which produced
// its factor) and after everything the caller queued on st before this
// call (v); the caller's stream waits for it in phi0_finish.
phiq_status phi0_start(const phiq_plan_s* P, const double* v, double* out0, void* T2, void* T3, hipStream_t st) {
  phiq_handle h = P->h;
  PHIQ_HIP(hipEventRecord(P->fork2, st));
  PHIQ_HIP(hipStreamWaitEvent(h->aux, P->fork2, 0));
  PHIQ_TRY(phi0_chain(P, v, out0, T2, T3, h->aux, true));
  PHIQ_HIP(hipEventRecord(P->phi0, h->aux));
  return PHIQ_OK;
}
phiq_status phi0_finish(const phiq_plan_s* P, hipStream_t st) {
  PHIQ_HIP(hipStreamWaitEvent(st, P->phi0, 0));
  return PHIQ_OK;
}

// l modified-squaring steps (eq. squaring) starting from y in Ycur (p x N);
// the last step writes into dst_final.
phiq_status squaring(const phiq_plan_s* P, double* Ycur, double* Yother, double* dst_final, void* T0, void* T1,
                     hipStream_t st) {
  const long long N = P->N;
  double* cur = Ycur;
  PHIQ_TRY(wait_join(P, st));
  for (int k = 0; k < P->l; ++k) {
    double* E[PHIQ_MAX_DIM];
    long long es[PHIQ_MAX_DIM];
    for (int d = 0; d < P->D; ++d) {
      E[d] = P->Esq[d] + (size_t)k * P->n[d] * P->n[d];
      es[d] = 0;
    }
    Front f;
    PHIQ_TRY(chain_front(P, cur, N, E, es, P->p, T0, T1, st, &f));
    double* dst = (k == P->l - 1) ? dst_final : (cur == Ycur ? Yother : Ycur);
    TtmArgs a = final_args(P, E[0], 0, f, P->p);
    a.O = dst;
    a.os = N;
    a.Yprev = cur;
    a.yps = N;
    PHIQ_TRY(L_ttm(P->h, K_TTM_SQUARE, a, P->opt.precision, st, &P->twins));
    cur = dst;
  }
  return PHIQ_OK;
}

// Device bytes of the intermediate tensors of one Gauss-rule execution:
// two node batches (max(m + 1, p) tensors each) and two p-vector squaring
// iterates.
size_t gauss_ws_bytes(const phiq_plan_s* P) {
  const long long N = P->N;
  const int nb = std::max(P->m + 1, P->p);
  const size_t tbytes = (P->D > 1 ? (size_t)nb * N * tensor_elem(P) : 0);
  const size_t ybytes = (size_t)P->p * N * sizeof(double);
  return 2 * align_up(tbytes) + 2 * align_up(ybytes);
}

// ws (nullable): a caller-provided workspace of ws_cap bytes used instead of
// the handle's (no allocation; PHIQ_ERR_OOM when it is too small).
phiq_status execute_gauss(phiq_plan P, const double* v, double* out, hipStream_t st, void* ws = nullptr,
                          size_t ws_cap = 0) {
  phiq_handle h = P->h;
  const long long N = P->N;
  const int p = P->p;
  const int nb = std::max(P->m + 1, p);
  const size_t tbytes = (P->D > 1 ? (size_t)nb * N * tensor_elem(P) : 0);
  const size_t ybytes = (size_t)p * N * sizeof(double);
  const size_t need = gauss_ws_bytes(P);
  char* wb;
  if (ws) {
    if (need > ws_cap) return PHIQ_ERR_OOM;
    wb = (char*)ws;
  } else {
    PHIQ_TRY(ensure(h, h->ws, std::max<size_t>(need, kAlign)));
    wb = (char*)h->ws.p;
  }
  void* T0 = wb;
  void* T1 = wb + align_up(tbytes);
  double* Ya = (double*)(wb + 2 * align_up(tbytes));
  double* Yb = (double*)(wb + 2 * align_up(tbytes) + align_up(ybytes));

  if (p == 0) return phi0_chain(P, v, out, T0, T1, st);

  // quadrature: the m node chains and the phi_0 chain as one batch per mode
  // product.  phi_0's factor exp(-tA^d) is slot m of the node tables (the
  // end of the scaling chain, joined here), so its first products ride in
  // the node batch instead of two launches on one vector (on a side stream
  // beside the node chains, phi_0 saved no time and slowed the launches it
  // overlapped).
  double* E[PHIQ_MAX_DIM];
  long long es[PHIQ_MAX_DIM];
  for (int d = 0; d < P->D; ++d) {
    E[d] = P->Enode[d];
    es[d] = (long long)P->n[d] * P->n[d];
  }
  PHIQ_TRY(wait_join(P, st));
  Front f;
  PHIQ_TRY(chain_front(P, v, 0, E, es, P->m + 1, T0, T1, st, &f));
  double* Y = (P->l == 0) ? out + N : Ya;
  for (int j0 = 0; j0 < p; j0 += 4) {
    TtmArgs a = final_args(P, P->Enode[0], es[0], f, P->m);
    a.coef = P->coef + (size_t)j0 * P->ldcoef;
    a.ldcoef = P->ldcoef;
    a.np = std::min(4, p - j0);
    a.Y = Y + (size_t)j0 * N;
    a.ys = N;
    PHIQ_TRY(L_ttm(P->h, K_TTM_ACCUM, a, P->opt.precision, st, &P->twins));
  }
  {  // phi_0 = (exp(-tA^0) (x) exp(-tA^1) ...) v: the last product of slot m,
     // before the squaring reuses the front's buffers
    Front f0 = f;
    f0.X = elem_offset(f.X, (long long)P->m * f.xs, f.f32);
    TtmArgs a = final_args(P, P->Ephi0[0], 0, f0, 1);
    a.O = out;
    a.os = 0;
    PHIQ_TRY(L_ttm(P->h, K_TTM_STORE, a, P->opt.precision, st, &P->twins));
  }
  if (P->l > 0) PHIQ_TRY(squaring(P, Ya, Yb, out + N, T0, T1, st));
  return PHIQ_OK;
}

// ---- int8 digit products (PHIQ_PREC_INT8) -----------------------------------
// Every chain starts from digits of its FP64 input (one exponent per tensor,
// from its max norm); the products over axes D-1..1 write digits of their
// output with an exponent raised by the bound ||e^{-cA^d}||_inf <= e^{c mu_d}
// (no reduction needed), the product over axis 0 writes FP64: the node
// outputs, summed by the node-sum kernel, or the squaring combination.
inline int i8_digits(double tol) { return tol >= 1e-6 ? 5 : (tol >= 1e-9 ? 6 : 7); }
inline int i8_delta(const phiq_plan_s* P, int d, double c) {
  return (int)std::ceil(c * P->mu[d] * 1.4426950408889634 + 1e-9);
}

struct I8Work {
  int S;
  int8_t* Enode[PHIQ_MAX_DIM];
  int8_t* Esq[PHIQ_MAX_DIM];
  int8_t* Ephi0[PHIQ_MAX_DIM];
  int* enode[PHIQ_MAX_DIM];
  int* esq[PHIQ_MAX_DIM];
  int* ephi0[PHIQ_MAX_DIM];
  int8_t* In;   // digits of the chain inputs (up to p tensors)
  int8_t* T[2]; // intermediate digits, nb tensors each
  int* ein;
  int* et[2];
  double* partial;
  int nbx;
};

// mode products over axes D-1..0 of the nb chains whose inputs are the
// digits `in` (shared when in_shared) with factors F[d] (fstride[d] rows per
// batch, 0 = one factor for all, plane stride fsp[d]); the last product runs
// with `last` (mode and FP64 output fields).
phiq_status i8_chain(const phiq_plan_s* P, const I8Work& w, const int8_t* in, const int* ein, bool in_shared,
                     int8_t* const* F, int* const* Fe, const long long* fsp, const long long* fstride,
                     const double* cfac, int nb, I8Args last, int last_mode, hipStream_t st) {
  const long long N = P->N;
  const int8_t* cur = in;
  const int* ce = ein;
  bool shared = in_shared;
  int pp = 0;
  for (int s = 0; s + 1 < P->D; ++s) {
    const int d = P->D - 1 - s;
    I8Args a{};
    a.S = w.S;
    a.E = F[d];
    a.es = fstride[d] * P->n[d];
    a.esp = fsp[d];
    a.ee = Fe[d];
    a.ees = fstride[d];
    a.delta = i8_delta(P, d, cfac[d]);
    a.X = cur;
    a.xs = shared ? 0 : (long long)w.S * N;
    a.xsp = N;
    a.xe = ce;
    a.xes = shared ? 0 : 1;
    a.M = a.K = P->n[d];
    a.L = N / P->n[d];
    a.nbatch = nb;
    a.O8 = w.T[pp];
    a.os8 = (long long)w.S * N;
    a.osp8 = N;
    a.oe = w.et[pp];
    double fl = 2.0 * a.M * a.K * (double)a.L * nb, by = (double)w.S * N * (shared ? 1 + nb : 2 * nb);
    PHIQ_TRY(prof_launch(P->h, st, K_TTM_STORE, fl, by, [&] { return launch_i8_product(a, kI8Slice, st); }));
    cur = w.T[pp];
    ce = w.et[pp];
    shared = false;
    pp ^= 1;
  }
  I8Args a = last;
  a.S = w.S;
  a.E = F[0];
  a.es = fstride[0] * P->n[0];
  a.esp = fsp[0];
  a.ee = Fe[0];
  a.ees = fstride[0];
  a.X = cur;
  a.xs = shared ? 0 : (long long)w.S * N;
  a.xsp = N;
  a.xe = ce;
  a.xes = shared ? 0 : 1;
  a.M = a.K = P->n[0];
  a.L = N / P->n[0];
  a.nbatch = nb;
  double f = 1.0;
  for (int k = 0; k <= PHIQ_MAX_P; ++k) {
    a.ifact[k] = 1.0 / f;
    f *= (k + 1);
  }
  const int cls = last_mode == kI8Square ? K_TTM_SQUARE : K_TTM_STORE;
  double fl = 2.0 * a.M * a.K * (double)a.L * nb, by = (double)w.S * N * (shared ? 1 : nb) + 8.0 * N * nb;
  return prof_launch(P->h, st, cls, fl, by, [&] { return launch_i8_product(a, last_mode, st); });
}

phiq_status execute_gauss_i8(phiq_plan P, const double* v, double* out, hipStream_t st) {
  phiq_handle h = P->h;
  const long long N = P->N;
  const int p = P->p, m = P->m, l = P->l, D = P->D;
  const int S = i8_digits(P->tol);
  const int nb = std::max(std::max(m, p), 1);
  // workspace: factor digits and exponents, input / intermediate digits,
  // node outputs (FP64), y ping-pong, partial maxima, tensor exponents
  size_t off = 0;
  auto take = [&](size_t bytes) {
    const size_t o = off;
    off += align_up(bytes);
    return o;
  };
  size_t oEn[PHIQ_MAX_DIM], oEs[PHIQ_MAX_DIM], oEp[PHIQ_MAX_DIM], oen[PHIQ_MAX_DIM], oes[PHIQ_MAX_DIM],
      oep[PHIQ_MAX_DIM];
  for (int d = 0; d < D; ++d) {
    const size_t nn = (size_t)P->n[d] * P->n[d];
    oEn[d] = take(nn * std::max(m, 1) * S);
    oEs[d] = take(nn * std::max(l, 1) * S);
    oEp[d] = take(nn * S);
    oen[d] = take(sizeof(int) * P->n[d] * std::max(m, 1));
    oes[d] = take(sizeof(int) * P->n[d] * std::max(l, 1));
    oep[d] = take(sizeof(int) * P->n[d]);
  }
  const int nbx = 256;
  const size_t oIn = take((size_t)S * N * std::max(p, 1));
  const size_t oT0 = take((size_t)S * N * nb);
  const size_t oT1 = take((size_t)S * N * nb);
  const size_t oV = take(sizeof(double) * N * std::max(m, 1));
  const size_t oYa = take(sizeof(double) * N * std::max(p, 1));
  const size_t oYb = take(sizeof(double) * N * std::max(p, 1));
  const size_t oPart = take(sizeof(double) * nbx * std::max(p, 1));
  const size_t oEx = take(sizeof(int) * 3 * (nb + 1));
  PHIQ_TRY(ensure(h, h->ws, std::max<size_t>(off, kAlign)));
  char* wb = (char*)h->ws.p;
  I8Work w{};
  w.S = S;
  for (int d = 0; d < D; ++d) {
    w.Enode[d] = (int8_t*)(wb + oEn[d]);
    w.Esq[d] = (int8_t*)(wb + oEs[d]);
    w.Ephi0[d] = (int8_t*)(wb + oEp[d]);
    w.enode[d] = (int*)(wb + oen[d]);
    w.esq[d] = (int*)(wb + oes[d]);
    w.ephi0[d] = (int*)(wb + oep[d]);
  }
  w.In = (int8_t*)(wb + oIn);
  w.T[0] = (int8_t*)(wb + oT0);
  w.T[1] = (int8_t*)(wb + oT1);
  double* V = (double*)(wb + oV);
  double* Ya = (double*)(wb + oYa);
  double* Yb = (double*)(wb + oYb);
  w.partial = (double*)(wb + oPart);
  w.nbx = nbx;
  w.ein = (int*)(wb + oEx);
  w.et[0] = w.ein + (nb + 1);
  w.et[1] = w.et[0] + (nb + 1);

  // digits of every factor (the squaring chain and phi_0 factors come from the side stream)
  PHIQ_TRY(wait_join(P, st));
  auto slice_rows = [&](const double* E, long long rows, int nd, int8_t* planes, int* ex) {
    return prof_launch(h, st, K_SLICE, 0.0, (8.0 + S) * rows * nd,
                       [&] { return launch_i8_slice_rows(E, rows, nd, S, planes, ex, st); });
  };
  auto slice_tensors = [&](const double* X, int nt, int8_t* planes, int* ex) {
    return prof_launch(h, st, K_SLICE, 0.0, (16.0 + S) * (double)N * nt, [&] {
      return launch_i8_slice_tensors(X, N, N, nt, S, w.partial, nbx, planes, (long long)S * N, ex, st);
    });
  };
  for (int d = 0; d < D; ++d) {
    const int nd = P->n[d];
    if (m > 0 && p > 0) PHIQ_TRY(slice_rows(P->Enode[d], (long long)m * nd, nd, w.Enode[d], w.enode[d]));
    if (l > 0) PHIQ_TRY(slice_rows(P->Esq[d], (long long)l * nd, nd, w.Esq[d], w.esq[d]));
    PHIQ_TRY(slice_rows(P->Ephi0[d], nd, nd, w.Ephi0[d], w.ephi0[d]));
  }
  PHIQ_TRY(slice_tensors(v, 1, w.In, w.ein));

  long long fsp[PHIQ_MAX_DIM], fstride[PHIQ_MAX_DIM];
  double cfac[PHIQ_MAX_DIM];
  // phi_0 = e^{-tA} v
  {
    int8_t* F[PHIQ_MAX_DIM];
    int* Fe[PHIQ_MAX_DIM];
    for (int d = 0; d < D; ++d) {
      F[d] = w.Ephi0[d];
      Fe[d] = w.ephi0[d];
      fsp[d] = (long long)P->n[d] * P->n[d];
      fstride[d] = 0;
      cfac[d] = P->t;
    }
    I8Args last{};
    last.O = out;
    last.os = 0;
    PHIQ_TRY(i8_chain(P, w, w.In, w.ein, true, F, Fe, fsp, fstride, cfac, 1, last, kI8Store, st));
  }
  if (p == 0) return PHIQ_OK;
  // quadrature: the m node chains on the shared input, node outputs in V
  {
    int8_t* F[PHIQ_MAX_DIM];
    int* Fe[PHIQ_MAX_DIM];
    for (int d = 0; d < D; ++d) {
      F[d] = w.Enode[d];
      Fe[d] = w.enode[d];
      fsp[d] = (long long)m * P->n[d] * P->n[d];
      fstride[d] = P->n[d];
      cfac[d] = std::ldexp(P->t, -l);  // (1 - theta) 2^{-l} t <= 2^{-l} t
    }
    I8Args last{};
    last.O = V;
    last.os = N;
    PHIQ_TRY(i8_chain(P, w, w.In, w.ein, true, F, Fe, fsp, fstride, cfac, m, last, kI8Store, st));
    double* Y = (l == 0) ? out + N : Ya;
    NodeSegs segs{};
    segs.V[0] = V;
    segs.count[0] = m;
    segs.nseg = 1;
    PHIQ_TRY(prof_launch(h, st, K_TTM_ACCUM, 0.0, 8.0 * N * (m + p),
                         [&] { return launch_node_sum(segs, N, P->coef, P->ldcoef, p, Y, st); }));
  }
  // modified squaring
  double* cur = Ya;
  for (int k = 0; k < l; ++k) {
    PHIQ_TRY(slice_tensors(cur, p, w.In, w.ein));
    int8_t* F[PHIQ_MAX_DIM];
    int* Fe[PHIQ_MAX_DIM];
    for (int d = 0; d < D; ++d) {
      const long long nn = (long long)P->n[d] * P->n[d];
      F[d] = w.Esq[d] + (size_t)k * nn;
      Fe[d] = w.esq[d] + (size_t)k * P->n[d];
      fsp[d] = (long long)l * nn;
      fstride[d] = 0;
      cfac[d] = std::ldexp(P->t, k - l);
    }
    double* dst = (k == l - 1) ? out + N : (cur == Ya ? Yb : Ya);
    I8Args last{};
    last.O = dst;
    last.os = N;
    last.Yprev = cur;
    last.yps = N;
    PHIQ_TRY(i8_chain(P, w, w.In, w.ein, false, F, Fe, fsp, fstride, cfac, p, last, kI8Square, st));
    cur = dst;
  }
  return PHIQ_OK;
}

// The l squaring steps of a linear combination (R23) on y_1..y_pe in cur
// (other: the second buffer of the pair); the last step forms y_pe only and
// writes it into out, or adds it when out already holds phi_0 b_0 (on the
// side stream when side is set).
phiq_status combo_squaring(const phiq_plan_s* P, double* cur, double* other, int pe, double* out, bool have_out,
                           bool side, void* T0, void* T1, hipStream_t st) {
  phiq_handle h = P->h;
  const long long N = P->N;
  PHIQ_TRY(wait_join(P, st));
  for (int k = 0; k < P->l; ++k) {
    double* Ek[PHIQ_MAX_DIM];
    long long e0[PHIQ_MAX_DIM];
    for (int d = 0; d < P->D; ++d) {
      Ek[d] = P->Esq[d] + (size_t)k * P->n[d] * P->n[d];
      e0[d] = 0;
    }
    const bool last = (k == P->l - 1);
    Front f;
    if (!last) {
      PHIQ_TRY(chain_front(P, cur, N, Ek, e0, pe, T0, T1, st, &f));
      double* dst = other;
      TtmArgs a = final_args(P, Ek[0], 0, f, pe);
      a.O = dst;
      a.os = N;
      a.Yprev = cur;
      a.yps = N;
      PHIQ_TRY(L_ttm(h, K_TTM_SQUARE, a, P->opt.precision, st, &P->twins));
      other = cur;
      cur = dst;
      continue;
    }
    PHIQ_TRY(chain_front(P, cur + (size_t)(pe - 1) * N, 0, Ek, e0, 1, T0, T1, st, &f));
    TtmArgs a = final_args(P, Ek[0], 0, f, 1);
    a.O = out;
    a.os = 0;
    a.Yprev = cur;
    a.yps = N;
    a.order0 = pe - 1;
    if (side) PHIQ_TRY(phi0_finish(P, st));
    a.yacc = have_out ? 1 : 0;
    PHIQ_TRY(L_ttm(h, K_TTM_SQUARE, a, P->opt.precision, st, &P->twins));
  }
  return PHIQ_OK;
}

// ---- linear combinations sum_j phi_j(Z) b_j, Z = -tA ------------------------
// The remark after Algorithm 2 writes sum_{j>=1} phi_j(Z) b_j as one integral
// of e^{(1-theta) Z} against the forcing g(theta) = sum_j theta^{j-1}/(j-1)! b_j.
// Scaling and squaring for it: x(s) = sum_j s^j phi_j(sZ) b_j solves
// x' = Z x + g(s), x(0) = 0, and x(2s) = e^{sZ} x(s) + (the same problem over
// [0, s] with g shifted by s), so the doubling needs the solutions for the
// forcings shifted by 0..p-1 places, X_i(s) = sum_k s^k phi_k(sZ) b_{k+i}:
//   X_i(2s) = e^{sZ} X_i(s) + sum_{r=0}^{p-1-i} s^r/r! X_{i+r}(s).
// With y_k = X_{p-k}(s) / s^k this is exactly eq. squaring (the modified
// squaring of y_1..y_p), so the squaring kernels are reused unchanged; the
// result is y_p at s = 1.  At s = 2^{-l} the node sum gives, per vector b_j,
//   y_{p-j+k} += 2^{l(p-j)} sum_q w_q theta_q^{k-1}/(k-1)! e^{(1-theta_q) s Z} b_j,
// k = 1..j: the usual node coefficients with a power-of-two factor.  Only y_p
// is needed after the last step, so that step applies one chain.
phiq_status execute_combo(phiq_plan P, const double* const* b, double* out, hipStream_t st) {
  phiq_handle h = P->h;
  const long long N = P->N;
  int pe = 0;  // highest order with a vector
  for (int j = 1; j <= P->p; ++j)
    if (b[j]) pe = j;
  const int nb = std::max(P->m + 1, P->p);
  const size_t tbytes = (P->D > 1 ? (size_t)nb * N * sizeof(double) : 0);
  const size_t ybytes = (size_t)std::max(1, P->p) * N * sizeof(double);
  const size_t t1bytes = (P->D > 1 ? (size_t)N * sizeof(double) : 0);
  const size_t need = 2 * align_up(tbytes) + 2 * align_up(ybytes) + 2 * align_up(t1bytes);
  PHIQ_TRY(ensure(h, h->ws, std::max<size_t>(need, kAlign)));
  char* wb = (char*)h->ws.p;
  void* T0 = wb;
  void* T1 = wb + align_up(tbytes);
  double* Ya = (double*)(wb + 2 * align_up(tbytes));
  double* Yb = (double*)(wb + 2 * align_up(tbytes) + align_up(ybytes));
  void* T2 = wb + 2 * align_up(tbytes) + 2 * align_up(ybytes);
  void* T3 = (char*)T2 + align_up(t1bytes);

  if (pe == 0) return phi0_chain(P, b[0], out, T0, T1, st);
  // phi_0 b_0 into out first: on the side stream when the squaring follows
  const bool side = b[0] && P->has_join && P->l > 0;
  bool have_out = false;
  if (b[0]) {
    if (side) {
      PHIQ_TRY(phi0_start(P, b[0], out, T2, T3, st));
    } else {
      PHIQ_TRY(phi0_chain(P, b[0], out, T0, T1, st));
    }
    have_out = true;
  }

  double* E[PHIQ_MAX_DIM];
  long long es[PHIQ_MAX_DIM];
  for (int d = 0; d < P->D; ++d) {
    E[d] = P->Enode[d];
    es[d] = (long long)P->n[d] * P->n[d];
  }
  // node sums, highest order first so that it writes every y_k
  for (int j = pe; j >= 1; --j) {
    if (!b[j]) continue;
    Front f;
    PHIQ_TRY(chain_front(P, b[j], 0, E, es, P->m, T0, T1, st, &f));
    if (P->l == 0) {  // only y_pe = sum_j phi_j(Z) b_j, straight into out
      TtmArgs a = final_args(P, P->Enode[0], es[0], f, P->m);
      a.coef = P->coef + (size_t)(j - 1) * P->ldcoef;
      a.ldcoef = P->ldcoef;
      a.np = 1;
      a.Y = out;
      a.ys = N;
      a.yacc = have_out ? 1 : 0;
      PHIQ_TRY(L_ttm(h, K_TTM_ACCUM, a, P->opt.precision, st, &P->twins));
      have_out = true;
      continue;
    }
    for (int k0 = 0; k0 < j; k0 += 4) {
      TtmArgs a = final_args(P, P->Enode[0], es[0], f, P->m);
      a.coef = P->coef + (size_t)k0 * P->ldcoef;
      a.ldcoef = P->ldcoef;
      a.np = std::min(4, j - k0);
      a.cexp = P->l * (pe - j);
      a.Y = Ya + (size_t)(pe - j + k0) * N;
      a.ys = N;
      a.yacc = (j == pe) ? 0 : 1;
      PHIQ_TRY(L_ttm(h, K_TTM_ACCUM, a, P->opt.precision, st, &P->twins));
    }
  }
  if (P->l == 0) return PHIQ_OK;
  return combo_squaring(P, Ya, Yb, pe, out, have_out, side, T0, T1, st);
}

// ---- adaptive Clenshaw-Curtis (Algorithm 2) --------------------------------
// Level 0 holds the 7 nodes j = 0..6 of the rule with n = 3 (2n+1 points);
// level k >= 1 holds the 3*2^k new (odd-j) nodes of the rule with n = 3*2^k.
void cc_level_nodes(int level, std::vector<double>& theta) {
  theta.clear();
  if (level == 0) {
    for (int j = 0; j <= 6; ++j) theta.push_back(0.5 * (1.0 + std::cos(M_PI * j / 6.0)));
  } else {
    const int n2 = 6 << level;  // 2n for this level
    for (int j = 1; j < n2; j += 2) theta.push_back(0.5 * (1.0 + std::cos(M_PI * (double)j / n2)));
  }
}

phiq_status cc_ensure_level(phiq_plan P, int level, hipStream_t st) {
  phiq_handle h = P->h;
  while ((int)P->cc_E.size() <= level) {
    const int lv = (int)P->cc_E.size();
    std::vector<double> theta;
    cc_level_nodes(lv, theta);
    const int cnt = (int)theta.size();
    size_t bytes = 0;
    for (int d = 0; d < P->D; ++d) bytes += align_up((size_t)cnt * P->n[d] * P->n[d] * sizeof(double));
    const size_t fp64_bytes = bytes;
    const bool lp = twin_prec(P->opt.precision);
    if (lp) bytes += twin_bytes(fp64_bytes / sizeof(double));
    DevBuf b;
    if (P->tr_slot >= 0) {
      // transient plan (phiq_action): the slot's table, reused call after call
      // (the slot's previous user finished before this call's upload)
      auto& pool = h->tr_cc[P->tr_slot];
      if ((int)pool.size() <= lv) pool.resize(lv + 1);
      PHIQ_TRY(ensure(h, pool[lv], bytes));
      b = pool[lv];
      P->cc_pooled = true;
    } else {
      if (h->cap_bytes && h->held() + bytes > h->cap_bytes) return PHIQ_ERR_OOM;
      if (hipMalloc(&b.p, bytes) != hipSuccess) {
        (void)hipGetLastError();
        return PHIQ_ERR_OOM;
      }
      b.cap = bytes;
    }
    P->cc_E.push_back(b);
    P->cc_count.push_back(cnt);
    std::vector<ExpTarget> tg;
    size_t o = 0;
    for (int d = 0; d < P->D; ++d) {
      const size_t nn = (size_t)P->n[d] * P->n[d];
      double* dd = (double*)((char*)b.p + o);
      for (int q = 0; q < cnt; ++q) tg.push_back({d, 1.0 - theta[q], dd + q * nn, q});
      o += align_up((size_t)cnt * nn * sizeof(double));
    }
    JobBlob blob;
    ExpmJobs ej;
    build_taylor_and_sigma(P, tg, blob, ej);
    if (blob.bytes.size() > P->jobs_cap) return PHIQ_ERR_UNSUPPORTED;
    int slot;
    void* hp;
    PHIQ_TRY(stage_acquire(h, blob.bytes.size(), &slot, &hp));
    std::memcpy(hp, blob.bytes.data(), blob.bytes.size());
    PHIQ_TRY(stage_copy(h, slot, P->jobs, blob.bytes.size(), st));
    PHIQ_TRY(run_taylor_sigma(P, P->jobs, ej, st));
    if (lp) {
      const size_t cnt64 = fp64_bytes / sizeof(double);
      char* tb = (char*)b.p + fp64_bytes;
      P->twins.t.push_back({(const double*)b.p, cnt64, tb, tb + cnt64 * 2});
      PHIQ_HIP(launch_convert((const double*)b.p, (long long)cnt64, P->opt.precision, tb, tb + cnt64 * 2, st));
    }
  }
  return PHIQ_OK;
}

double* cc_level_E(const phiq_plan_s* P, int level, int d) {
  size_t o = 0;
  for (int e = 0; e < d; ++e) o += align_up((size_t)P->cc_count[level] * P->n[e] * P->n[e] * sizeof(double));
  return (double*)((char*)P->cc_E[level].p + o);
}

// Stopping tolerance of Algorithm 2.  With lower-precision mode products the
// successive approximations differ by their rounding noise, so the test is
// floored at a level that noise stays under (2^-18 for FP32 products,
// 2^-12 for split bf16).
double cc_tolerance(const phiq_plan_s* P) {
  if (P->opt.precision == PHIQ_PREC_FP32) return std::max(P->tol, std::ldexp(1.0, -18));
  if (P->opt.precision == PHIQ_PREC_BF16X3) return std::max(P->tol, std::ldexp(1.0, -12));
  return P->tol;
}

phiq_status execute_cc(phiq_plan P, const double* v, double* out, hipStream_t st, phiq_report* rep) {
  phiq_handle h = P->h;
  const long long N = P->N;
  const int p = P->p;
  const int cap = P->opt.cc_max_doublings;
  const int maxcnt = 3 * (1 << cap) + 1;
  const int nb = std::max(std::max(maxcnt, 7), p);
  const size_t tbytes = (P->D > 1 ? (size_t)nb * N * tensor_elem(P) : 0);
  const size_t ybytes = (size_t)p * N * sizeof(double);
  PHIQ_TRY(ensure(h, h->ws, 2 * align_up(tbytes) + 2 * align_up(ybytes) + kAlign));
  char* wb = (char*)h->ws.p;
  void* T0 = wb;
  void* T1 = wb + align_up(tbytes);
  double* Ya = (double*)(wb + 2 * align_up(tbytes));
  double* Yb = (double*)(wb + 2 * align_up(tbytes) + align_up(ybytes));
  if (p == 0) return phi0_chain(P, v, out, T0, T1, st);

  const int nblk = 256;
  PHIQ_TRY(ensure(h, h->partial, (size_t)nblk * PHIQ_MAX_P * 2 * sizeof(double)));
  if (!h->partial_host) {
    if (hipHostMalloc((void**)&h->partial_host, (size_t)nblk * PHIQ_MAX_P * 2 * sizeof(double),
                      hipHostMallocDefault) != hipSuccess) {
      h->partial_host = nullptr;
      return PHIQ_ERR_OOM;
    }
  }

  // per-level device decisions, their pinned host copies and events
  const int nlev = cap + 1;
  PHIQ_TRY(ensure(h, h->cc_ctl, (size_t)(nlev + 1) * sizeof(CcCtl)));
  if (!h->cc_ctl_host) {
    if (hipHostMalloc((void**)&h->cc_ctl_host, 16 * sizeof(CcCtl), hipHostMallocDefault) != hipSuccess) {
      h->cc_ctl_host = nullptr;
      return PHIQ_ERR_OOM;
    }
  }
  while ((int)h->cc_ev.size() < nlev + 1) {
    hipEvent_t e = nullptr;
    PHIQ_HIP(hipEventCreateWithFlags(&e, hipEventDisableTiming));
    h->cc_ev.push_back(e);
  }
  CcCtl* ctl = (CcCtl*)h->cc_ctl.p;
  double* ybuf[2] = {Ya, Yb};

  // One level of Algorithm 2: the node vectors of its new nodes, the node sum
  // over every stored node with the weights of the level's rule, and (from
  // level 1 on) the relative change, decided on the device and copied to the
  // host.  guard (nullable): when the flag is set on the device, the level's
  // products, node sum and change test do nothing.
  auto run_level = [&](int level, const int* guard) -> phiq_status {
    PHIQ_TRY(cc_ensure_level(P, level, st));
    const int cnt = P->cc_count[level];
    if ((int)h->cc_levels.size() <= level) h->cc_levels.resize(level + 1);
    PHIQ_TRY(ensure(h, h->cc_levels[level], (size_t)cnt * N * sizeof(double)));
    double* V = (double*)h->cc_levels[level].p;
    // node vectors v_i = e^{(1 - x_i) A} b of this level (Algorithm 2, step 2)
    double* E[PHIQ_MAX_DIM];
    long long es[PHIQ_MAX_DIM];
    for (int d = 0; d < P->D; ++d) {
      E[d] = cc_level_E(P, level, d);
      es[d] = (long long)P->n[d] * P->n[d];
    }
    h->guard = guard;
    Front f;
    phiq_status sf = chain_front(P, v, 0, E, es, cnt, T0, T1, st, &f);
    if (sf == PHIQ_OK) {
      TtmArgs a = final_args(P, E[0], es[0], f, cnt);
      a.O = V;
      a.os = N;
      sf = L_ttm(P->h, K_TTM_STORE, a, P->opt.precision, st, &P->twins);
    }
    h->guard = nullptr;
    PHIQ_TRY(sf);
    // weights of the full (2n+1)-point rule, n = 3*2^level, in storage order
    const int n2 = 6 << level;
    std::vector<double> xt(n2 + 1), wt(n2 + 1);
    clenshaw_curtis(n2 + 1, xt.data(), wt.data());
    std::vector<int> ord;  // rule index of every stored node
    NodeSegs segs{};
    for (int lv = 0; lv <= level; ++lv) {
      if (lv == 0) {
        for (int j = 0; j <= 6; ++j) ord.push_back(j << level);
      } else {
        for (int j = 1; j < (6 << lv); j += 2) ord.push_back(j << (level - lv));
      }
      segs.V[lv] = (const double*)h->cc_levels[lv].p;
      segs.count[lv] = P->cc_count[lv];
    }
    segs.nseg = level + 1;
    const int total = (int)ord.size();
    int slot;
    void* hp;
    PHIQ_TRY(stage_acquire(h, sizeof(double) * (size_t)p * total, &slot, &hp));
    double* hc = (double*)hp;
    for (int j = 0; j < p; ++j) {
      double fact = 1.0;
      for (int k = 2; k <= j; ++k) fact *= k;
      for (int i = 0; i < total; ++i) hc[(size_t)j * total + i] = wt[ord[i]] * std::pow(xt[ord[i]], j) / fact;
    }
    PHIQ_TRY(stage_copy(h, slot, P->coef, sizeof(double) * (size_t)p * total, st));
    // y_j = sum_i w_i x_i^{j-1}/(j-1)! v_i (Algorithm 2, step 3)
    double* ynew = ybuf[level % 2];
    PHIQ_TRY(prof_launch(h, st, K_NODE_SUM, 2.0 * p * total * (double)N, 8.0 * (total + p) * (double)N,
                         [&] { return launch_node_sum(segs, N, P->coef, total, p, ynew, st, guard); }));
    if (level > 0) {
      // err = max_j ||y_j - y~_j||_inf / ||y_j||_inf (Algorithm 2, step 4)
      double* yold = ybuf[(level - 1) % 2];
      PHIQ_TRY(prof_launch(h, st, K_ABSDIFF, 2.0 * p * (double)N, 16.0 * p * (double)N, [&] {
        return launch_absdiff_max(ynew, yold, p, N, (double*)h->partial.p, nblk, st, guard);
      }));
      PHIQ_HIP(launch_cc_decide((const double*)h->partial.p, nblk, p, cc_tolerance(P), guard, ctl + level, st));
      PHIQ_HIP(hipMemcpyAsync(h->cc_ctl_host + level, ctl + level, sizeof(CcCtl), hipMemcpyDeviceToHost, st));
      PHIQ_HIP(hipEventRecord(h->cc_ev[level], st));
    }
    return PHIQ_OK;
  };

  // Levels 0 and 1 always run.  Then, before the host reads level k's
  // decision, level k + 1 is already enqueued behind a guard on that
  // decision: the GPU works on it while the host waits, and after
  // convergence its launches return at once.
  PHIQ_TRY(run_level(0, nullptr));
  PHIQ_TRY(run_level(1, nullptr));
  double err = INFINITY;
  int level = 1;
  bool converged = false;
  for (;; ++level) {
    if (level < cap) PHIQ_TRY(run_level(level + 1, &ctl[level].stop));
    PHIQ_HIP(hipEventSynchronize(h->cc_ev[level]));
    err = h->cc_ctl_host[level].err;
    if (h->cc_ctl_host[level].stop) {
      converged = true;
      break;
    }
    if (level >= cap) break;
  }
  double* ycur = ybuf[level % 2];
  if (rep) {
    rep->m = (6 << level) + 1;
    rep->cc_doublings = level;
    rep->cc_err = err;
  }
  if (!converged) return PHIQ_ERR_NOT_CONVERGED;
  if (P->l > 0) {
    double* other = (ycur == Ya) ? Yb : Ya;
    PHIQ_TRY(squaring(P, ycur, other, out + N, T0, T1, st));
  } else {
    PHIQ_HIP(hipMemcpyAsync(out + N, ycur, (size_t)p * N * sizeof(double), hipMemcpyDeviceToDevice, st));
  }
  return phi0_chain(P, v, out, T0, T1, st);
}

// Sum_j phi_j(-tA) b_j with the adaptive Clenshaw-Curtis rule (Algorithm 2
// on the linear combination of R23).  Each level stores the node vectors
// e^{(1 - x_i) s Z} b_j of every vector b_j; after each level the base sums
//   y_{pe-j+k} = sum_j 2^{l(pe-j)} sum_i w_i x_i^{k-1}/(k-1)! e^{(1-x_i) s Z} b_j
// (k = 1..j) are formed over all stored nodes with the weights of the level's
// rule, one node-sum launch per vector (the running y_1..y_pe enter the next
// launch as inputs with coefficient 1), and the doubling stops when the
// largest relative change of y_1..y_pe is below the tolerance.  Then the
// squaring of the Gauss form.
phiq_status execute_combo_cc(phiq_plan P, const double* const* b, double* out, hipStream_t st, phiq_report* rep) {
  phiq_handle h = P->h;
  const long long N = P->N;
  const int cap = P->opt.cc_max_doublings;
  int pe = 0;
  std::vector<int> js;  // orders with a vector, highest first
  for (int j = P->p; j >= 1; --j)
    if (b[j]) js.push_back(j);
  if (!js.empty()) pe = js[0];
  const int nbj = (int)js.size();
  const int maxcnt = 3 * (1 << cap) + 1;
  const int nb = std::max(std::max(maxcnt, 7), P->p);
  const size_t tbytes = (P->D > 1 ? (size_t)nb * N * sizeof(double) : 0);
  const size_t ybytes = (size_t)std::max(1, P->p) * N * sizeof(double);
  PHIQ_TRY(ensure(h, h->ws, 2 * align_up(tbytes) + 2 * align_up(ybytes) + kAlign));
  char* wb = (char*)h->ws.p;
  void* T0 = wb;
  void* T1 = wb + align_up(tbytes);
  double* Ya = (double*)(wb + 2 * align_up(tbytes));
  double* Yb = (double*)(wb + 2 * align_up(tbytes) + align_up(ybytes));

  // phi_0 b_0 into out first (this stream)
  const bool have_out = b[0] != nullptr;
  if (have_out) PHIQ_TRY(phi0_chain(P, b[0], out, T0, T1, st));
  if (pe == 0) return PHIQ_OK;

  const int nblk = 256;
  PHIQ_TRY(ensure(h, h->partial, (size_t)nblk * PHIQ_MAX_P * 2 * sizeof(double)));
  if (!h->partial_host) {
    if (hipHostMalloc((void**)&h->partial_host, (size_t)nblk * PHIQ_MAX_P * 2 * sizeof(double),
                      hipHostMallocDefault) != hipSuccess) {
      h->partial_host = nullptr;
      return PHIQ_ERR_OOM;
    }
  }
  double* ycur = Ya;
  double* ynew = Yb;
  double err = INFINITY;
  int level = 0;
  bool converged = false;
  for (;; ++level) {
    PHIQ_TRY(cc_ensure_level(P, level, st));
    const int cnt = P->cc_count[level];
    if ((int)h->cc_levels.size() <= level) h->cc_levels.resize(level + 1);
    PHIQ_TRY(ensure(h, h->cc_levels[level], (size_t)nbj * cnt * N * sizeof(double)));
    double* E[PHIQ_MAX_DIM];
    long long es[PHIQ_MAX_DIM];
    for (int d = 0; d < P->D; ++d) {
      E[d] = cc_level_E(P, level, d);
      es[d] = (long long)P->n[d] * P->n[d];
    }
    // this level's node vectors of every b_j (Algorithm 2, step 2)
    for (int q = 0; q < nbj; ++q) {
      Front f;
      PHIQ_TRY(chain_front(P, b[js[q]], 0, E, es, cnt, T0, T1, st, &f));
      TtmArgs a = final_args(P, E[0], es[0], f, cnt);
      a.O = (double*)h->cc_levels[level].p + (size_t)q * cnt * N;
      a.os = N;
      PHIQ_TRY(L_ttm(h, K_TTM_STORE, a, P->opt.precision, st, &P->twins));
    }
    // weights of the full (2n+1)-point rule, n = 3*2^level, in storage order
    const int n2 = 6 << level;
    std::vector<double> xt(n2 + 1), wt(n2 + 1);
    clenshaw_curtis(n2 + 1, xt.data(), wt.data());
    std::vector<int> ord;  // rule index of every stored node
    for (int lv = 0; lv <= level; ++lv) {
      if (lv == 0) {
        for (int j = 0; j <= 6; ++j) ord.push_back(j << level);
      } else {
        for (int j = 1; j < (6 << lv); j += 2) ord.push_back(j << (level - lv));
      }
    }
    const int total = (int)ord.size();
    // coefficient blocks, one per vector: pe rows x (pe identity columns for
    // the running sums, except in the first) + total node columns
    std::vector<size_t> boff(nbj);
    size_t ncoef = 0;
    for (int q = 0; q < nbj; ++q) {
      boff[q] = ncoef;
      ncoef += (size_t)pe * ((q ? pe : 0) + total);
    }
    PHIQ_TRY(ensure(h, h->combo_coef, ncoef * sizeof(double)));
    int slot;
    void* hp;
    PHIQ_TRY(stage_acquire(h, ncoef * sizeof(double), &slot, &hp));
    double* hc = (double*)hp;
    for (int q = 0; q < nbj; ++q) {
      const int j = js[q], id = q ? pe : 0, ld = id + total;
      const double scale = std::ldexp(1.0, P->l * (pe - j));
      double* c = hc + boff[q];
      for (int r = 0; r < pe; ++r) {
        for (int col = 0; col < id; ++col) c[(size_t)r * ld + col] = (col == r) ? 1.0 : 0.0;
        const int k = r - (pe - j);  // y_{r+1} takes theta^k / k! of b_j when 0 <= k < j
        double fact = 1.0;
        for (int i = 2; i <= k; ++i) fact *= i;
        for (int i = 0; i < total; ++i)
          c[(size_t)r * ld + id + i] = (k >= 0) ? scale * wt[ord[i]] * std::pow(xt[ord[i]], k) / fact : 0.0;
      }
    }
    PHIQ_TRY(stage_copy(h, slot, h->combo_coef.p, ncoef * sizeof(double), st));
    // y_1..y_pe over all stored nodes (Algorithm 2, step 3)
    for (int q = 0; q < nbj; ++q) {
      NodeSegs segs{};
      int ns = 0;
      if (q) {
        segs.V[ns] = ynew;
        segs.count[ns++] = pe;
      }
      for (int lv = 0; lv <= level; ++lv) {
        segs.V[ns] = (const double*)h->cc_levels[lv].p + (size_t)q * P->cc_count[lv] * N;
        segs.count[ns++] = P->cc_count[lv];
      }
      segs.nseg = ns;
      const double* cq = (const double*)h->combo_coef.p + boff[q];
      const int ld = (q ? pe : 0) + total;
      PHIQ_TRY(prof_launch(h, st, K_NODE_SUM, 2.0 * pe * ld * (double)N, 8.0 * (ld + pe) * (double)N,
                           [&] { return launch_node_sum(segs, N, cq, ld, pe, ynew, st); }));
    }
    if (level > 0) {
      // err = max_k ||y_k - y~_k||_inf / ||y_k||_inf (Algorithm 2, step 4)
      PHIQ_TRY(prof_launch(h, st, K_ABSDIFF, 2.0 * pe * (double)N, 16.0 * pe * (double)N, [&] {
        return launch_absdiff_max(ynew, ycur, pe, N, (double*)h->partial.p, nblk, st);
      }));
      PHIQ_HIP(hipMemcpyAsync(h->partial_host, h->partial.p, (size_t)nblk * pe * 2 * sizeof(double),
                              hipMemcpyDeviceToHost, st));
      PHIQ_HIP(hipStreamSynchronize(st));
      err = 0.0;
      for (int j = 0; j < pe; ++j) {
        double num = 0.0, den = 0.0;
        for (int bk = 0; bk < nblk; ++bk) {
          num = std::max(num, h->partial_host[((size_t)bk * pe + j) * 2 + 0]);
          den = std::max(den, h->partial_host[((size_t)bk * pe + j) * 2 + 1]);
        }
        err = std::max(err, den > 0 ? num / den : num);
      }
    }
    std::swap(ycur, ynew);
    if (level > 0 && err <= cc_tolerance(P)) {
      converged = true;
      break;
    }
    if (level >= cap) break;
  }
  if (rep) {
    rep->m = (6 << level) + 1;
    rep->cc_doublings = level;
    rep->cc_err = err;
  }
  if (!converged) return PHIQ_ERR_NOT_CONVERGED;
  if (P->l > 0) return combo_squaring(P, ycur, ycur == Ya ? Yb : Ya, pe, out, have_out, false, T0, T1, st);
  // l = 0: out (+)= y_pe
  NodeSegs segs{};
  int ns = 0;
  if (have_out) {
    segs.V[ns] = out;
    segs.count[ns++] = 1;
  }
  segs.V[ns] = ycur + (size_t)(pe - 1) * N;
  segs.count[ns++] = 1;
  segs.nseg = ns;
  int slot;
  void* hp;
  PHIQ_TRY(stage_acquire(h, 2 * sizeof(double), &slot, &hp));
  ((double*)hp)[0] = ((double*)hp)[1] = 1.0;
  PHIQ_TRY(ensure(h, h->combo_coef, 2 * sizeof(double)));
  PHIQ_TRY(stage_copy(h, slot, h->combo_coef.p, 2 * sizeof(double), st));
  return prof_launch(h, st, K_NODE_SUM, 2.0 * ns * (double)N, 8.0 * (ns + 1) * (double)N, [&] {
    return launch_node_sum(segs, N, (const double*)h->combo_coef.p, ns, 1, out, st);
  });
}

}  // namespace

// ---------------------------------------------------------------------------
// C ABI
// ---------------------------------------------------------------------------
extern "C" {

const char* phiq_status_string(phiq_status s) {
  switch (s) {
    case PHIQ_OK: return "PHIQ_OK";
    case PHIQ_ERR_INVALID_ARG: return "PHIQ_ERR_INVALID_ARG";
    case PHIQ_ERR_NONFINITE: return "PHIQ_ERR_NONFINITE";
    case PHIQ_ERR_NOT_CONVERGED: return "PHIQ_ERR_NOT_CONVERGED";
    case PHIQ_ERR_OOM: return "PHIQ_ERR_OOM";
    case PHIQ_ERR_HIP: return "PHIQ_ERR_HIP";
    case PHIQ_ERR_UNSUPPORTED: return "PHIQ_ERR_UNSUPPORTED";
  }
  return "PHIQ_UNKNOWN_STATUS";
}

phiq_status phiq_options_default(phiq_options* o) {
  if (!o) return PHIQ_ERR_INVALID_ARG;
  std::memset(o, 0, sizeof(*o));
  o->rule = PHIQ_RULE_GAUSS;
  o->precision = PHIQ_PREC_FP64;
  o->l = -1;
  o->m = -1;
  o->alpha = -1.0;
  o->c1 = 0.0;
  o->c2 = 1.0;
  o->cc_max_doublings = 6;
  o->workspace_cap = 0;
  o->use_graphs = 0;
  o->selector = PHIQ_SEL_PAPER;
  o->slab_products = 0;
  return PHIQ_OK;
}

phiq_status phiq_create(phiq_handle* out, int device) {
  if (!out) return PHIQ_ERR_INVALID_ARG;
  int count = 0;
  if (hipGetDeviceCount(&count) != hipSuccess) {
    (void)hipGetLastError();
    return PHIQ_ERR_HIP;
  }
  if (device < 0 || device >= count) return PHIQ_ERR_INVALID_ARG;
  {
    // the fixed array of phiq_plan_execute_noalloc: its address on this device
    DeviceGuard g(device);
    PHIQ_TRY(noalloc_scratch_init(device));
  }
  phiq_handle h = new (std::nothrow) phiq_handle_s;
  if (!h) return PHIQ_ERR_OOM;
  h->device = device;
  *out = h;
  return PHIQ_OK;
}

phiq_status phiq_destroy(phiq_handle h) {
  if (!h) return PHIQ_ERR_INVALID_ARG;
  DeviceGuard g(h->device);
  (void)hipDeviceSynchronize();
  if (h->ws.p) (void)hipFree(h->ws.p);
  if (h->scratch.p) (void)hipFree(h->scratch.p);
  if (h->partial.p) (void)hipFree(h->partial.p);
  if (h->cc_ctl.p) (void)hipFree(h->cc_ctl.p);
  if (h->cc_ctl_host) (void)hipHostFree(h->cc_ctl_host);
  for (hipEvent_t e : h->cc_ev)
    if (e) (void)hipEventDestroy(e);
  if (h->combo_coef.p) (void)hipFree(h->combo_coef.p);
  for (auto& b : h->cc_levels)
    if (b.p) (void)hipFree(b.p);
  if (h->partial_host) (void)hipHostFree(h->partial_host);
  if (h->batch.p) (void)hipFree(h->batch.p);
  for (auto e : h->prof.pool) (void)hipEventDestroy(e);
  if (h->tr_fork) (void)hipEventDestroy(h->tr_fork);
  if (h->tr_join) (void)hipEventDestroy(h->tr_join);
  for (auto& g : h->graphs) (void)hipGraphExecDestroy(g.exec);
  if (h->aux) (void)hipStreamDestroy(h->aux);
  if (h->ps) (void)hipStreamDestroy(h->ps);
  if (h->tr_ready) (void)hipEventDestroy(h->tr_ready);
  if (h->copy) (void)hipStreamDestroy(h->copy);
  if (h->tr_fork2) (void)hipEventDestroy(h->tr_fork2);
  if (h->tr_phi0) (void)hipEventDestroy(h->tr_phi0);
  for (int k = 0; k < 2; ++k) {
    if (h->tr_buf[k].p) (void)hipFree(h->tr_buf[k].p);
    for (auto& b : h->tr_cc[k])
      if (b.p) (void)hipFree(b.p);
    if (h->tr_free[k]) (void)hipEventDestroy(h->tr_free[k]);
    if (h->tr_up[k]) (void)hipEventDestroy(h->tr_up[k]);
  }
  for (int k = 0; k < 3; ++k) {
    if (h->stage.host[k]) (void)hipHostFree(h->stage.host[k]);
    if (h->stage.ev[k]) (void)hipEventDestroy(h->stage.ev[k]);
  }
  delete h;
  return PHIQ_OK;
}

phiq_status phiq_plan_create(phiq_handle h, const phiq_kron_op* op, double t, int p, double tol,
                             const phiq_options* opt, phiq_plan* plan, phiq_report* rep, hipStream_t stream) {
  if (!h || !plan) return PHIQ_ERR_INVALID_ARG;
  DeviceGuard g(h->device);
  if (opt && opt->workspace_cap) h->cap_bytes = opt->workspace_cap;
  return plan_build(h, op, t, p, tol, opt, false, plan, rep, stream);
}

phiq_status phiq_plan_execute(phiq_plan plan, const double* v, int nrhs, double* out, phiq_report* rep,
                              hipStream_t stream) {
  if (!plan || !v || !out || nrhs < 1) return PHIQ_ERR_INVALID_ARG;
  const long long N = plan->N;
  // v and out must not overlap
  const char* vb = (const char*)v;
  const char* ve = vb + (size_t)nrhs * N * sizeof(double);
  const char* ob = (const char*)out;
  const char* oe = ob + (size_t)nrhs * (plan->p + 1) * N * sizeof(double);
  if (vb < oe && ob < ve) return PHIQ_ERR_INVALID_ARG;
  DeviceGuard g(plan->h->device);
  for (int r = 0; r < nrhs; ++r) {
    const double* vr = v + (size_t)r * N;
    double* outr = out + (size_t)r * (plan->p + 1) * N;
    if (plan->opt.precision == PHIQ_PREC_INT8) {
      PHIQ_TRY(execute_gauss_i8(plan, vr, outr, stream));
    } else if (plan->opt.rule == PHIQ_RULE_GAUSS) {
      PHIQ_TRY(execute_gauss(plan, vr, outr, stream));
    } else {
      PHIQ_TRY(execute_cc(plan, vr, outr, stream, rep));
    }
  }
  if (rep) {
    rep->l = plan->l;
    if (plan->opt.rule == PHIQ_RULE_GAUSS) rep->m = plan->m;
    rep->alpha = plan->alpha;
    rep->log10_bound = plan->log10_bound;
    rep->selector = plan->selector;
    const int chains_per = (plan->p > 0 ? rep->m + plan->l * plan->p : 0) + 1;
    rep->ttm_chains = chains_per * nrhs;
    rep->workspace_bytes = plan->h->held();
    rep->precision_floor = precision_floor(plan->opt.precision);
    rep->tol_met = plan->tol >= rep->precision_floor;
  }
  return PHIQ_OK;
}

phiq_status phiq_plan_execute_combo(phiq_plan plan, const double* const* b, double* out, hipStream_t stream) {
  if (!plan || !b || !out) return PHIQ_ERR_INVALID_ARG;
  if (plan->opt.precision == PHIQ_PREC_INT8) return PHIQ_ERR_UNSUPPORTED;
  // (Clenshaw-Curtis: a plan's doubling cap is at most 10, so the node sums
  // take at most 11 levels plus the running sums: the 12 segments of NodeSegs)
  const long long N = plan->N;
  const char* ob = (const char*)out;
  const char* oe = ob + (size_t)N * sizeof(double);
  int pe = -1;
  for (int j = 0; j <= plan->p; ++j) {
    if (!b[j]) continue;
    pe = j;
    const char* vb = (const char*)b[j];
    const char* ve = vb + (size_t)N * sizeof(double);
    if (vb < oe && ob < ve) return PHIQ_ERR_INVALID_ARG;  // out must not overlap an input
  }
  if (pe < 0) return PHIQ_ERR_INVALID_ARG;
  // the node coefficients are scaled by up to 2^{l (pe - 1)}
  if (pe > 1 && (long long)plan->l * (pe - 1) > 900) return PHIQ_ERR_UNSUPPORTED;
  DeviceGuard g(plan->h->device);
  if (plan->opt.rule == PHIQ_RULE_CC) return execute_combo_cc(plan, b, out, stream, nullptr);
  return execute_combo(plan, b, out, stream);
}

phiq_status phiq_plan_destroy(phiq_plan plan) {
  if (!plan) return PHIQ_ERR_INVALID_ARG;
  DeviceGuard g(plan->h->device);
  if (!plan->transient && plan->mem) {
    // plan memory may still be read by queued work
    (void)hipDeviceSynchronize();
  }
  if (!plan->cc_E.empty() && !plan->cc_pooled) (void)hipDeviceSynchronize();
  delete plan;
  return PHIQ_OK;
}

phiq_status phiq_action(phiq_handle h, const phiq_kron_op* op, double t, int p, const double* v, double tol,
                        const phiq_options* opt, double* out, phiq_report* rep, hipStream_t stream) {
  if (!h || !v || !out) return PHIQ_ERR_INVALID_ARG;
  DeviceGuard g(h->device);
  if (opt && opt->workspace_cap) h->cap_bytes = opt->workspace_cap;
  phiq_plan P = nullptr;
  phiq_report r{};
  const bool want_graph = (!opt || opt->use_graphs) && !h->prof.on;
  // Without graphs, the plan (upload, 1D exponentials) goes on the handle's
  // plan stream and the caller's stream waits for it: the next call's plan
  // then runs while this call's quadrature and squaring do.
  hipStream_t pst = stream;
  if (!want_graph) {
    if (!h->ps) PHIQ_HIP(hipStreamCreateWithFlags(&h->ps, hipStreamNonBlocking));
    if (!h->tr_ready) PHIQ_HIP(hipEventCreateWithFlags(&h->tr_ready, hipEventDisableTiming));
    for (int k = 0; k < 2; ++k)
      if (!h->tr_free[k]) PHIQ_HIP(hipEventCreateWithFlags(&h->tr_free[k], hipEventDisableTiming));
    pst = h->ps;
    // the plan stream must not start before what the caller queued earlier
    // on its stream that the plan could depend on: nothing (the plan reads
    // only host data and its own buffer), so no wait here
  }
  PHIQ_TRY(plan_build(h, op, t, p, tol, opt, true, &P, &r, pst, /*defer_device=*/true));
  phiq_status s = PHIQ_OK;
  const bool graphable = want_graph && P->opt.rule == PHIQ_RULE_GAUSS && P->opt.precision != PHIQ_PREC_INT8;
  if (graphable) {
    // v and out must not overlap (checked by execute on the eager path)
    const char* vb = (const char*)v;
    const char* ob = (const char*)out;
    const size_t nb = (size_t)P->N * sizeof(double);
    if (vb < ob + (P->p + 1) * nb && ob < vb + nb) {
      delete P;
      return PHIQ_ERR_INVALID_ARG;
    }
    std::vector<long long> key = {(long long)(uintptr_t)P->mem, (long long)P->bytes, (long long)(uintptr_t)v,
                                  (long long)(uintptr_t)out, (long long)(uintptr_t)h->ws.p, (long long)h->ws.cap,
                                  (long long)(uintptr_t)stream, P->opt.precision, P->D, P->p, P->l, P->m, P->K,
                                  P->has_join ? 1 : 0};
    for (int d = 0; d < P->D; ++d) {
      key.push_back(P->n[d]);
      key.push_back(P->sigma[d]);
    }
    hipGraphExec_t exec = nullptr;
    for (const auto& g : h->graphs)
      if (g.key == key) exec = g.exec;
    bool was_seen = false;
    for (const auto& k : h->seen)
      if (k == key) was_seen = true;
    if (exec) {
      P->has_join = (P->l > 0);
      if (hipGraphLaunch(exec, stream) != hipSuccess) s = PHIQ_ERR_HIP;
    } else if (was_seen) {
      hipGraph_t graph = nullptr;
      P->single_stream = true;  // a linear graph: no side-stream branches
      s = hipStreamBeginCapture(stream, hipStreamCaptureModeRelaxed) == hipSuccess ? PHIQ_OK : PHIQ_ERR_HIP;
      phiq_status se = PHIQ_OK;
      if (s == PHIQ_OK) {
        se = plan_enqueue(P, stream);
        if (se == PHIQ_OK) se = execute_gauss(P, v, out, stream);
        if (hipStreamEndCapture(stream, &graph) != hipSuccess) s = PHIQ_ERR_HIP;
      }
      if (s == PHIQ_OK && se == PHIQ_OK && graph &&
          hipGraphInstantiate(&exec, graph, nullptr, nullptr, 0) == hipSuccess) {
        if (h->graphs.size() >= 16) {
          (void)hipGraphExecDestroy(h->graphs.front().exec);
          h->graphs.erase(h->graphs.begin());
        }
        h->graphs.push_back({key, exec});
        if (hipGraphLaunch(exec, stream) != hipSuccess) s = PHIQ_ERR_HIP;
      } else {
        (void)hipGetLastError();
        s = PHIQ_ERR_HIP;
      }
      if (graph) (void)hipGraphDestroy(graph);
      if (s != PHIQ_OK || se != PHIQ_OK) {
        // capture failed: fall back to the eager launches for this call
        s = plan_enqueue(P, stream);
        if (s == PHIQ_OK) s = phiq_plan_execute(P, v, 1, out, &r, stream);
      }
    } else {
      s = plan_enqueue(P, stream);
      if (s == PHIQ_OK) s = phiq_plan_execute(P, v, 1, out, &r, stream);
      if (s == PHIQ_OK) {
        if (h->seen.size() >= 64) h->seen.erase(h->seen.begin());
        h->seen.push_back(key);
      }
    }
    if (rep) {
      r.l = P->l;
      r.m = P->m;
      r.alpha = P->alpha;
      r.log10_bound = P->log10_bound;
      r.ttm_chains = (P->p > 0 ? P->m + P->l * P->p : 0) + 1;
      r.workspace_bytes = h->held();
    }
  } else {
    s = plan_enqueue(P, pst);
    if (s == PHIQ_OK && pst != stream) {
      if (hipEventRecord(h->tr_ready, pst) != hipSuccess || hipStreamWaitEvent(stream, h->tr_ready, 0) != hipSuccess)
        s = PHIQ_ERR_HIP;
    }
    if (s == PHIQ_OK) s = phiq_plan_execute(P, v, 1, out, &r, stream);
  }
  if (P->tr_slot >= 0 && h->tr_free[P->tr_slot]) {
    if (hipEventRecord(h->tr_free[P->tr_slot], stream) == hipSuccess) h->tr_used[P->tr_slot] = true;
  }
  if (rep) *rep = r;
  if (!P->cc_E.empty() && !P->cc_pooled) (void)hipStreamSynchronize(stream);
  delete P;  // transient: memory stays in the handle
  return s;
}

phiq_status phiq_kron_apply(phiq_handle h, int dim, const int* n, const double* const* F, const double* x, double* y,
                            int nvec, phiq_precision prec, hipStream_t stream) {
  if (!h || !n || !F || !x || !y || nvec < 1 || dim < 1 || dim > PHIQ_MAX_DIM) return PHIQ_ERR_INVALID_ARG;
  if (prec != PHIQ_PREC_FP64 && prec != PHIQ_PREC_FP32 && prec != PHIQ_PREC_BF16X3) return PHIQ_ERR_INVALID_ARG;
  long long N = 1;
  for (int d = 0; d < dim; ++d) {
    if (n[d] < 1 || n[d] > PHIQ_MAX_N || !F[d]) return PHIQ_ERR_INVALID_ARG;
    N *= n[d];
  }
  const char* xb = (const char*)x;
  const char* xe = xb + (size_t)nvec * N * sizeof(double);
  const char* yb = (const char*)y;
  const char* ye = yb + (size_t)nvec * N * sizeof(double);
  if (xb < ye && yb < xe) return PHIQ_ERR_INVALID_ARG;
  DeviceGuard g(h->device);
  const int lp = prec != PHIQ_PREC_FP64;
  const size_t tb = align_up((size_t)nvec * N * (lp ? sizeof(float) : sizeof(double)));
  PHIQ_TRY(ensure(h, h->ws, dim > 1 ? 2 * tb : kAlign));
  void* T[2] = {h->ws.p, (char*)h->ws.p + tb};
  TwinMap tw;
  if (lp) {
    size_t need = 0;
    for (int d = 0; d < dim; ++d) need += twin_bytes((size_t)n[d] * n[d]);
    PHIQ_TRY(ensure(h, h->scratch, need));
    char* c = (char*)h->scratch.p;
    for (int d = 0; d < dim; ++d) {
      const size_t cnt = (size_t)n[d] * n[d];
      tw.t.push_back({F[d], cnt, c, c + cnt * 2});
      PHIQ_HIP(launch_convert(F[d], (long long)cnt, prec, c, c + cnt * 2, stream));
      c += twin_bytes(cnt);
    }
  }
  const void* cur = x;
  int cur_f32 = 0;
  for (int s = 0; s < dim; ++s) {
    const int d = dim - 1 - s;
    TtmArgs a{};
    a.E = F[d];
    a.es = 0;
    a.X = cur;
    a.xs = N;
    a.x_f32 = cur_f32;
    a.O = (s == dim - 1) ? (void*)y : T[s % 2];
    a.o_f32 = (s == dim - 1) ? 0 : lp;
    a.os = N;
    a.M = a.K = n[d];
    a.L = (int)(N / n[d]);
    a.nbatch = nvec;
    PHIQ_TRY(L_ttm(h, K_TTM_STORE, a, prec, stream, &tw));
    cur = a.O;
    cur_f32 = a.o_f32;
  }
  return PHIQ_OK;
}

phiq_status phiq_expm(phiq_handle h, int n, int nmat, const double* X, const double* xnorm, double* E,
                      hipStream_t stream) {
  if (!h || !X || !xnorm || !E || n < 1 || n > PHIQ_MAX_N || nmat < 1 || nmat > 4096) return PHIQ_ERR_INVALID_ARG;
  const size_t nn = (size_t)n * n;
  const char* xb = (const char*)X;
  const char* xe = xb + nmat * nn * sizeof(double);
  const char* eb = (const char*)E;
  const char* ee = eb + nmat * nn * sizeof(double);
  if (xb < ee && eb < xe) return PHIQ_ERR_INVALID_ARG;
  double nu = 0.0;
  std::vector<int> sig(nmat);
  for (int b = 0; b < nmat; ++b) {
    if (!std::isfinite(xnorm[b])) return PHIQ_ERR_NONFINITE;
    if (xnorm[b] < 0) return PHIQ_ERR_INVALID_ARG;
    int s = 0;
    while (std::ldexp(xnorm[b], -s) > kThetaMax) ++s;
    if (s > 1000) return PHIQ_ERR_INVALID_ARG;
    sig[b] = s;
    nu = std::max(nu, std::ldexp(xnorm[b], -s));
  }
  DeviceGuard g(h->device);
  const int K = taylor_degree(nu);
  int smax = 0;
  for (int b = 0; b < nmat; ++b) smax = std::max(smax, sig[b]);
  // scratch: powers K*nmat*nn, ping-pong 2*nmat*nn, jobs
  JobBlob blob;
  std::vector<ScaleJob> sj;
  Layout L;
  const size_t offZ = L.take(sizeof(double) * K * nmat * nn);
  const size_t offS0 = L.take(sizeof(double) * nmat * nn);
  const size_t offS1 = L.take(sizeof(double) * nmat * nn);
  const size_t offJ = L.take(1 << 20);
  PHIQ_TRY(ensure(h, h->scratch, L.off));
  char* base = (char*)h->scratch.p;
  double* Z = (double*)(base + offZ);
  double* S[2] = {(double*)(base + offS0), (double*)(base + offS1)};
  auto zpow = [&](int b, int k) { return Z + ((size_t)b * K + (k - 1)) * nn; };
  for (int b = 0; b < nmat; ++b) {
    ScaleJob s{};
    s.src = X + b * nn;
    s.dst = zpow(b, 1);
    s.s = std::ldexp(1.0, -sig[b]);
    s.n = n;
    sj.push_back(s);
  }
  const size_t o_scale = blob.add(sj);
  std::vector<std::pair<size_t, int>> rounds;
  for (int pw = 1; pw < K; pw *= 2) {
    std::vector<GemmJob> gj;
    for (int b = 0; b < nmat; ++b)
      for (int j = 1; j <= pw && j + pw <= K; ++j) gj.push_back(GemmJob{zpow(b, j), zpow(b, pw), zpow(b, j + pw), n, 0});
    rounds.push_back({blob.add(gj), (int)gj.size()});
  }
  std::vector<TaylorJob> tj;
  for (int b = 0; b < nmat; ++b) {
    TaylorJob j{};
    j.Zpow = zpow(b, 1);
    j.dst[0] = sig[b] > 0 ? S[0] + b * nn : E + b * nn;
    j.c[0] = 1.0;
    j.n = n;
    j.K = K;
    j.nt = 1;
    tj.push_back(j);
  }
  const size_t o_tay = blob.add(tj);
  std::vector<std::pair<size_t, int>> sq;
  for (int r = 1; r <= smax; ++r) {
    std::vector<GemmJob> gj;
    for (int b = 0; b < nmat; ++b) {
      if (sig[b] < r) continue;
      const double* src = S[(r - 1) % 2] + b * nn;
      gj.push_back(GemmJob{src, src, (r == sig[b]) ? E + b * nn : S[r % 2] + b * nn, n, 0});
    }
    sq.push_back({blob.add(gj), (int)gj.size()});
  }
  if (blob.bytes.size() > (1 << 20)) return PHIQ_ERR_UNSUPPORTED;
  int slot;
  void* hp;
  PHIQ_TRY(stage_acquire(h, blob.bytes.size(), &slot, &hp));
  std::memcpy(hp, blob.bytes.data(), blob.bytes.size());
  char* jd = base + offJ;
  PHIQ_TRY(stage_copy(h, slot, jd, blob.bytes.size(), stream));
  PHIQ_TRY(L_scale(h, (const ScaleJob*)(jd + o_scale), (int)sj.size(), n, stream));
  for (const auto& r : rounds) PHIQ_TRY(L_gemm(h, (const GemmJob*)(jd + r.first), r.second, n, stream));
  PHIQ_TRY(L_taylor(h, (const TaylorJob*)(jd + o_tay), (int)tj.size(), n, K, stream));
  for (const auto& r : sq) PHIQ_TRY(L_gemm(h, (const GemmJob*)(jd + r.first), r.second, n, stream));
  return PHIQ_OK;
}

phiq_status phiq_profile_start(phiq_handle h, unsigned class_mask) {
  if (!h) return PHIQ_ERR_INVALID_ARG;
  h->prof.mask = class_mask ? class_mask : ~0u;
  h->prof.recs.clear();
  h->prof.next = 0;
  h->prof.on = true;
  h->prof.open = true;
  return PHIQ_OK;
}

phiq_status phiq_profile_enable(phiq_handle h, int on) {
  if (!h || !h->prof.open) return PHIQ_ERR_INVALID_ARG;
  h->prof.on = on != 0;
  return PHIQ_OK;
}

phiq_status phiq_profile_stop(phiq_handle h, phiq_kernel_stat* stats, int max_stats, int* n_stats) {
  if (!h || (max_stats > 0 && !stats) || max_stats < 0) return PHIQ_ERR_INVALID_ARG;
  DeviceGuard g(h->device);
  h->prof.on = false;
  h->prof.open = false;
  PHIQ_HIP(hipDeviceSynchronize());
  phiq_kernel_stat agg[K_NCLASS];
  std::memset(agg, 0, sizeof(agg));
  for (int c = 0; c < K_NCLASS; ++c) std::strncpy(agg[c].name, kProfClass[c], sizeof(agg[c].name) - 1);
  for (const auto& r : h->prof.recs) {
    float ms = 0.f;
    if (hipEventElapsedTime(&ms, r.e0, r.e1) != hipSuccess) return PHIQ_ERR_HIP;
    agg[r.cls].launches += 1;
    agg[r.cls].ms += ms;
    agg[r.cls].flops += r.flops;
    agg[r.cls].bytes += r.bytes;
  }
  h->prof.recs.clear();
  h->prof.next = 0;
  int k = 0;
  for (int c = 0; c < K_NCLASS; ++c)
    if (agg[c].launches > 0) {
      if (k < max_stats) stats[k] = agg[c];
      ++k;
    }
  if (n_stats) *n_stats = std::min(k, max_stats);
  return PHIQ_OK;
}

phiq_status phiq_tile_config(phiq_handle h, int kind, int cfg, int* count) {
  if (!h || kind < 0 || kind > 4) return PHIQ_ERR_INVALID_ARG;
  const int nc = kind <= 2 ? ttm_num_configs(kind) : (kind == 3 ? bf16r_num_configs() : bf16r_square_num_configs());
  if (count) *count = nc;
  if (cfg < -1 || cfg >= nc) return PHIQ_ERR_INVALID_ARG;
  h->force_cfg[kind] = cfg;
  return PHIQ_OK;
}

phiq_status phiq_autotune(phiq_handle h, int dim, const int* n, int p, int m, double* times, hipStream_t st) {
  // times is [64][16] (ms per launch shape and tile shape)
  if (!h || !n || dim < 1 || dim > PHIQ_MAX_DIM || p < 0 || p > PHIQ_MAX_P || m < 1 || m > 4096)
    return PHIQ_ERR_INVALID_ARG;
  long long N = 1;
  for (int d = 0; d < dim; ++d) {
    if (n[d] < 1 || n[d] > PHIQ_MAX_N) return PHIQ_ERR_INVALID_ARG;
    N *= n[d];
  }
  DeviceGuard g(h->device);
  const int nbmax = std::max(m + 1, std::max(p, 1));
  const size_t tb = align_up((size_t)nbmax * N * sizeof(double));
  const size_t eb = align_up((size_t)nbmax * PHIQ_MAX_N * PHIQ_MAX_N / 16 * sizeof(double));
  size_t emax = 0;
  for (int d = 0; d < dim; ++d) emax = std::max(emax, (size_t)nbmax * n[d] * n[d] * sizeof(double));
  const size_t need = 2 * tb + align_up(emax) + align_up((size_t)4 * nbmax * sizeof(double));
  (void)eb;
  PHIQ_TRY(ensure(h, h->ws, need));
  char* wb = (char*)h->ws.p;
  PHIQ_HIP(hipMemsetAsync(wb, 0, need, st));
  double* X = (double*)wb;
  double* O = (double*)(wb + tb);
  double* E = (double*)(wb + 2 * tb);
  double* coef = (double*)(wb + 2 * tb + align_up(emax));
  hipEvent_t e0, e1;
  PHIQ_HIP(hipEventCreate(&e0));
  PHIQ_HIP(hipEventCreate(&e1));
  // the launch shapes of a phi-action: store (nodes + phi_0, and p RHS),
  // node sum, squaring; every axis in turn is the contracted one
  struct Shape {
    int kind, M, L, nb;
  };
  std::vector<Shape> shapes;
  for (int d = 0; d < dim; ++d) {
    const int L = (int)(N / n[d]);
    shapes.push_back({0, n[d], L, m + 1});  // node chains with phi_0's (Gauss)
    shapes.push_back({0, n[d], L, 1});  // phi_0
    if (p > 0 && p != m && p != 1) shapes.push_back({0, n[d], L, p});  // squaring orders
    if (d == 0 && p > 0) {
      shapes.push_back({1, n[d], L, m});
      shapes.push_back({2, n[d], L, p});
    }
  }
  int ti = 0;
  for (const auto& sh : shapes) {
    TtmArgs a{};
    a.E = E;
    a.es = 0;
    a.X = X;
    a.xs = N;
    a.O = O;
    a.os = N;
    a.M = a.K = sh.M;
    a.L = sh.L;
    a.nbatch = sh.nb;
    a.coef = coef;
    a.ldcoef = sh.nb;
    a.np = std::min(4, std::max(1, p));
    a.Y = O;
    a.ys = N;
    a.Yprev = X;
    a.yps = N;
    for (int k = 0; k <= PHIQ_MAX_P; ++k) a.ifact[k] = 1.0;
    int best = -1;
    float best_ms = 1e30f;
    for (int c = 0; c < ttm_num_configs(sh.kind); ++c) {
      if (launch_kind(sh.kind, a, PHIQ_PREC_FP64, st, c) != hipSuccess) continue;  // warm-up
      PHIQ_HIP(hipEventRecord(e0, st));
      const int reps = 3;
      for (int r = 0; r < reps; ++r)
        if (launch_kind(sh.kind, a, PHIQ_PREC_FP64, st, c) != hipSuccess) return PHIQ_ERR_HIP;
      PHIQ_HIP(hipEventRecord(e1, st));
      PHIQ_HIP(hipEventSynchronize(e1));
      float ms = 0.f;
      PHIQ_HIP(hipEventElapsedTime(&ms, e0, e1));
      ms /= reps;
      if (times && ti < 64 && c < 16) times[ti * 16 + c] = ms;
      if (ms < best_ms) {
        best_ms = ms;
        best = c;
      }
    }
    if (best >= 0) {
      const int nbk = sh.kind == 1 ? 1 : sh.nb;
      bool found = false;
      for (auto& e : h->tune)
        if (e.kind == sh.kind && e.M == sh.M && e.L == sh.L && e.nb == nbk) {
          e.cfg = best;
          found = true;
        }
      if (!found) h->tune.push_back({sh.kind, sh.M, sh.L, nbk, best});
    }
    ++ti;
  }
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  return PHIQ_OK;
}

}  // extern "C"

// ---- helpers for the batched entry point (batched.cpp) --------------------
namespace phiq {

phiq_status batch_arena(phiq_handle h, size_t bytes, void** dev) {
  PHIQ_TRY(ensure(h, h->batch, std::max<size_t>(bytes, kAlign)));
  *dev = h->batch.p;
  return PHIQ_OK;
}

phiq_status batch_stage(phiq_handle h, size_t bytes, int* slot, void** host) {
  return stage_acquire(h, bytes, slot, host);
}

phiq_status batch_fetch(phiq_handle h, int slot, void* dst, size_t bytes, hipStream_t st) {
  return stage_fetch(h, slot, dst, bytes, st);
}

phiq_status plan_settle(phiq_plan P) {
  if (!P) return PHIQ_ERR_INVALID_ARG;
  DeviceGuard g(P->h->device);
  if (P->has_join) PHIQ_HIP(hipEventSynchronize(P->join));
  P->has_join = false;
  return PHIQ_OK;
}

bool plan_profiling(phiq_plan P) { return P && P->h->prof.on; }

const float* handle_mlp(phiq_handle h) { return (h && !h->mlp.empty()) ? h->mlp.data() : nullptr; }

}  // namespace phiq

namespace phiq {
phiq_status plan_execute_in(phiq_plan P, const double* v, double* out, void* ws, size_t ws_cap, hipStream_t st,
                            size_t* need) {
  if (!P || !v || !out || !ws) return PHIQ_ERR_INVALID_ARG;
  if (P->opt.rule != PHIQ_RULE_GAUSS || P->opt.precision == PHIQ_PREC_INT8) return PHIQ_ERR_UNSUPPORTED;
  // live timing creates and records events per launch
  if (P->h->prof.on) return PHIQ_ERR_UNSUPPORTED;
  const long long N = P->N;
  const char* vb = (const char*)v;
  const char* ve = vb + (size_t)N * sizeof(double);
  const char* ob = (const char*)out;
  const char* oe = ob + (size_t)(P->p + 1) * N * sizeof(double);
  if (vb < oe && ob < ve) return PHIQ_ERR_INVALID_ARG;
  const size_t nd = gauss_ws_bytes(P);
  if (need) *need = nd;
  if (nd > ws_cap) return PHIQ_ERR_OOM;
  DeviceGuard g(P->h->device);
  return execute_gauss(P, v, out, st, ws, ws_cap);
}
int plan_device(phiq_plan P) { return P ? P->h->device : -1; }
}  // namespace phiq

extern "C" phiq_status phiq_selector_set(phiq_handle h, const float* w) {
  if (!h) return PHIQ_ERR_INVALID_ARG;
  if (!w) {
    h->mlp.clear();
    return PHIQ_OK;
  }
  for (int i = 0; i < kMlpParams; ++i)
    if (!std::isfinite(w[i])) return PHIQ_ERR_NONFINITE;
  h->mlp.assign(w, w + kMlpParams);
  return PHIQ_OK;
}

extern "C" phiq_status phiq_selector_load(phiq_handle h, const char* weights_path) {
  if (!h || !weights_path) return PHIQ_ERR_INVALID_ARG;
  FILE* f = std::fopen(weights_path, "rb");
  if (!f) return PHIQ_ERR_INVALID_ARG;
  std::vector<float> w(kMlpParams + 1);
  const size_t got = std::fread(w.data(), sizeof(float), w.size(), f);
  std::fclose(f);
  if (got != (size_t)kMlpParams) return PHIQ_ERR_INVALID_ARG;  // shorter or longer than one weight vector
  return phiq_selector_set(h, w.data());
}

namespace phiq {

}  // namespace phiq
