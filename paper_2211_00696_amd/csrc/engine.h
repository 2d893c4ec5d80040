// Shared internals of the phi-action engine: the handle and plan objects,
// the launch helpers and the chain / squaring drivers that every execution
// path uses.  Private to the library's host units:
//   plan.cpp      parameter selection, plan layout and build, 1D exponentials
//   launch.cpp    mode-product launches, live timing, workspace and staging
//   gauss.cpp     Kronecker chains, phi_0, the modified squaring, Gauss rule
//   int8.cpp      the int8-digit precision form
//   combo.cpp     linear combinations sum_j phi_j b_j (Gauss and CC)
//   cc.cpp        adaptive Clenshaw-Curtis (Algorithm 2)
//   autotune.cpp  tile autotuner, forced tile shapes, live-timing entry points
//   api.cpp       the C ABI entry points
#pragma once
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

int taylor_degree(double nu);
double infnorm(const double* A, int n);

}  // namespace phiq

// The C ABI's opaque objects live at global scope; they use the phiq types.
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
  int force_cfg[8] = {-1, -1, -1, -1, -1, -1, -1, -1};  // phiq_tile_config: one shape for every launch of a kind
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
  // Gauss, 1 <= p <= 4: the node-sum coefficients of a linear combination
  // with every b_1..b_p set, p x (p m): row q (y_{q+1}), column (p - j) m + i
  // (node i of b_j) holds 2^{l (p - j)} w_i theta_i^k / k!, k = q - (p - j),
  // zero where k < 0 (execute_combo's one-launch node sum)
  double* coefc = nullptr;
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
  std::vector<char> cc_valid;  // 0: the level's table was skipped on the device (recompute before use)
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

namespace phiq {

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

hipEvent_t prof_event(phiq_handle h);

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

// ---- launch.cpp ---------------------------------------------------------------
void ttm_work(const TtmArgs& a, int cls, double* flops, double* bytes);
int tuned_cfg(phiq_handle h, int kind, const TtmArgs& a);
int fallback_cfg(int kind, const TtmArgs& a);
int launch_kind(int kind, const TtmArgs& a, phiq_precision prec, hipStream_t st, int cfg);
inline int kind_of(int cls) { return cls == K_TTM_ACCUM ? 1 : (cls == K_TTM_SQUARE ? 2 : 0); }
phiq_status L_ttm(phiq_handle h, int cls, const TtmArgs& a0, phiq_precision prec, hipStream_t st,
                  const TwinMap* tw = nullptr);
phiq_status L_gemm(phiq_handle h, const GemmJob* jobs, int njobs, int nm, hipStream_t st);
phiq_status L_taylor(phiq_handle h, const TaylorJob* jobs, int njobs, int nm, int K, hipStream_t st);
phiq_status L_scale(phiq_handle h, const ScaleJob* jobs, int njobs, int nm, hipStream_t st);
phiq_status ensure(phiq_handle h, DevBuf& b, size_t bytes);
phiq_status stage_acquire(phiq_handle h, size_t bytes, int* slot, void** host);
phiq_status stage_copy(phiq_handle h, int slot, void* dst, size_t bytes, hipStream_t st);
phiq_status stage_fetch(phiq_handle h, int slot, void* dst, size_t bytes, hipStream_t st);

// ---- plan.cpp -----------------------------------------------------------------
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

void build_taylor_and_sigma(const phiq_plan_s* P, const std::vector<ExpTarget>& tg, JobBlob& blob,
                            ExpmJobs& ej);
void build_powers(const phiq_plan_s* P, JobBlob& blob, ExpmJobs& ej);
int nmax_of(const phiq_plan_s* P);
phiq_status run_taylor_sigma(const phiq_plan_s* P, const char* jobs_dev, const ExpmJobs& ej, hipStream_t st);
phiq_status convert_range(const phiq_plan_s* P, const double* E, size_t count, hipStream_t st);
phiq_status wait_join(const phiq_plan_s* P, hipStream_t st);
phiq_status plan_enqueue(phiq_plan P, hipStream_t st);
phiq_status plan_build(phiq_handle h, const phiq_kron_op* op, double t, int p, double tol, const phiq_options* uopt,
                       bool transient, phiq_plan* out, phiq_report* rep, hipStream_t st, bool defer_device = false);

// ---- gauss.cpp: chains, phi_0, squaring, the Gauss rule -----------------------
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

phiq_status chain_front(const phiq_plan_s* P, const double* X, long long xs, double* const* Ebase, long long const* es,
                        int nb, void* T0, void* T1, hipStream_t st, Front* f, bool beside = false, int group = 0,
                        const TtmSegs* segs = nullptr);
TtmArgs final_args(const phiq_plan_s* P, const double* E, long long es, const Front& f, int nb);
phiq_status phi0_chain(const phiq_plan_s* P, const double* v, double* out0, void* T0, void* T1, hipStream_t st,
                       bool side = false);
phiq_status phi0_start(const phiq_plan_s* P, const double* v, double* out0, void* T2, void* T3, hipStream_t st);
phiq_status phi0_finish(const phiq_plan_s* P, hipStream_t st);
phiq_status squaring(const phiq_plan_s* P, double* Ycur, double* Yother, double* dst_final, void* T0, void* T1,
                     hipStream_t st);
size_t gauss_ws_bytes(const phiq_plan_s* P, int g = 1);
int rhs_group(const phiq_plan_s* P, int nrhs);
phiq_status execute_gauss_group(phiq_plan P, const double* v, int g, double* out, hipStream_t st);
phiq_status execute_gauss(phiq_plan P, const double* v, double* out, hipStream_t st, void* ws = nullptr,
                          size_t ws_cap = 0);

// ---- int8.cpp, combo.cpp, cc.cpp ----------------------------------------------
phiq_status execute_gauss_i8(phiq_plan P, const double* v, double* out, hipStream_t st);
phiq_status combo_squaring(const phiq_plan_s* P, double* cur, double* other, int pe, double* out, bool have_out,
                           bool side, void* T0, void* T1, hipStream_t st);
phiq_status execute_combo(phiq_plan P, const double* const* b, double* out, hipStream_t st);
phiq_status execute_combo_cc(phiq_plan P, const double* const* b, double* out, hipStream_t st, phiq_report* rep);
void cc_level_nodes(int level, std::vector<double>& theta);
phiq_status cc_compute_level(phiq_plan P, int lv, hipStream_t st);
phiq_status cc_ensure_level(phiq_plan P, int level, hipStream_t st);
double* cc_level_E(const phiq_plan_s* P, int level, int d);
double cc_tolerance(const phiq_plan_s* P);
phiq_status execute_cc(phiq_plan P, const double* v, double* out, hipStream_t st, phiq_report* rep);

}  // namespace phiq
