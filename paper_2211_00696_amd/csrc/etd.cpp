// phiq_etdrk4: exponential time differencing of order 4 (Cox-Matthews) on
// top of the phi-function actions, with the repeated step replayed from a
// captured hipGraph.
//
// One step of u' = -A u + F(u), F(u) = c1 u + c3 u^3, with L = -A:
//   a  = e^{hL/2} u + h/2 phi_1(hL/2) F(u)
//   b  = e^{hL/2} u + h/2 phi_1(hL/2) F(a)
//   c  = e^{hL/2} a + h/2 phi_1(hL/2) (2 F(b) - F(u))
//   u <- e^{hL} u + h [f1 F(u) + 2 f2 (F(a) + F(b)) + f3 F(c)],
//   f1 = phi_1 - 3 phi_2 + 4 phi_3, f2 = phi_2 - 2 phi_3, f3 = -phi_2 + 4 phi_3.
// form 0: four plans serve every step: phi_0 and phi_0..1 at h/2, phi_0 and
// phi_0..3 at h; the last runs on the three vectors F(u), F(a)+F(b), F(c)
// in one execution.
// form 1: every stage is one linear combination sum_j phi_j b_j
// (phiq_plan_execute_combo): a, b and c with phi_0..1 at h/2, and the update
// with b_0 = u and the phi_1..3 vectors regrouped from f1, f2, f3.
#include <cmath>
#include <cstring>

#include <hip/hip_runtime_api.h>

#include "phiq_internal.h"

#define PHIQ_TRY(x)                  \
  do {                               \
    const phiq_status s_ = (x);      \
    if (s_ != PHIQ_OK) return s_;    \
  } while (0)
#define PHIQ_HIP(x)                  \
  do {                               \
    if ((x) != hipSuccess) {         \
      (void)hipGetLastError();       \
      return PHIQ_ERR_HIP;           \
    }                                \
  } while (0)

namespace phiq {
namespace {

struct EtdPlans {
  phiq_plan half0 = nullptr, half1 = nullptr, full0 = nullptr, full3 = nullptr;
  ~EtdPlans() {
    for (phiq_plan p : {half0, half1, full0, full3})
      if (p) phiq_plan_destroy(p);
  }
};

// Device buffers of one step (N doubles each unless noted).
struct EtdBufs {
  double* in2;   // 3N: F(u), F(a) + F(b), F(c)
  double* e_u;   // e^{hL/2} u
  double* p1u;   // 2N: phi_0, phi_1 (hL/2) F(u)
  double* a;
  double* fa;
  double* p1a;   // 2N: phi_0, phi_1 (hL/2) F(a)
  double* mix;   // 2 F(b) - F(u)
  double* e_a;   // e^{hL/2} a
  double* p1m;   // 2N: phi_0, phi_1 (hL/2) mix
  double* e_full;  // e^{hL} u
  double* g;     // 12N: phi_0..3 (hL) of the three vectors in in2
};
constexpr int kEtdBufN = 27;

phiq_status etd_step(const EtdPlans& P, const EtdBufs& B, double* u, double tau, double c1, double c3, long long N,
                     hipStream_t st) {
  const double hh = 0.5 * tau;
  double* fu = B.in2;
  double* fab = B.in2 + N;
  double* fc = B.in2 + 2 * N;
  PHIQ_HIP(launch_etd_nonlin(u, fu, N, c1, c3, st));
  PHIQ_TRY(phiq_plan_execute(P.half0, u, 1, B.e_u, nullptr, st));
  PHIQ_TRY(phiq_plan_execute(P.half1, fu, 1, B.p1u, nullptr, st));
  PHIQ_HIP(launch_etd_stage(B.e_u, B.p1u + N, hh, B.a, B.fa, N, c1, c3, st));
  PHIQ_TRY(phiq_plan_execute(P.half1, B.fa, 1, B.p1a, nullptr, st));
  PHIQ_HIP(launch_etd_stage_b(B.e_u, B.p1a + N, hh, fu, B.fa, B.mix, fab, N, c1, c3, st));
  PHIQ_TRY(phiq_plan_execute(P.half0, B.a, 1, B.e_a, nullptr, st));
  PHIQ_TRY(phiq_plan_execute(P.half1, B.mix, 1, B.p1m, nullptr, st));
  PHIQ_HIP(launch_etd_stage(B.e_a, B.p1m + N, hh, nullptr, fc, N, c1, c3, st));
  PHIQ_TRY(phiq_plan_execute(P.full0, u, 1, B.e_full, nullptr, st));
  PHIQ_TRY(phiq_plan_execute(P.full3, B.in2, 3, B.g, nullptr, st));
  PHIQ_HIP(launch_etd_final(B.e_full, B.g, tau, u, N, st));
  return PHIQ_OK;
}

// Buffers of the linear-combination form (N doubles each).
struct EtdComboBufs {
  double *fu, *fa, *fab, *s, *a, *b, *c, *b1, *b2, *b3, *unew;
};
constexpr int kEtdComboBufN = 11;

phiq_status etd_step_combo(const EtdPlans& P, const EtdComboBufs& B, double* u, double tau, double c1, double c3,
                           long long N, hipStream_t st) {
  const double hh = 0.5 * tau;
  PHIQ_HIP(launch_etd_cf_stage(u, B.fu, B.s, hh, N, c1, c3, st));
  {
    const double* b[2] = {u, B.s};  // a = e^{hL/2} u + phi_1(hL/2) (h/2) F(u)
    PHIQ_TRY(phiq_plan_execute_combo(P.half1, b, B.a, st));
  }
  PHIQ_HIP(launch_etd_cf_stage(B.a, B.fa, B.s, hh, N, c1, c3, st));
  {
    const double* b[2] = {u, B.s};  // b = e^{hL/2} u + phi_1(hL/2) (h/2) F(a)
    PHIQ_TRY(phiq_plan_execute_combo(P.half1, b, B.b, st));
  }
  PHIQ_HIP(launch_etd_cf_b(B.b, B.fu, B.fa, B.s, B.fab, hh, N, c1, c3, st));
  {
    const double* b[2] = {B.a, B.s};  // c = e^{hL/2} a + phi_1(hL/2) (h/2) (2 F(b) - F(u))
    PHIQ_TRY(phiq_plan_execute_combo(P.half1, b, B.c, st));
  }
  PHIQ_HIP(launch_etd_cf_final(B.c, B.fu, B.fab, B.b1, B.b2, B.b3, tau, N, c1, c3, st));
  {
    const double* b[4] = {u, B.b1, B.b2, B.b3};
    PHIQ_TRY(phiq_plan_execute_combo(P.full3, b, B.unew, st));
  }
  PHIQ_HIP(launch_etd_copy(B.unew, u, N, st));
  return PHIQ_OK;
}

// Kronecker chains of one phiq_plan_execute_combo with every b_j set.
int combo_chains(int p, int m, int l) { return 1 + p * m + (l > 0 ? p * (l - 1) + 1 : 0); }

struct GraphState {
  hipStream_t cs = nullptr;
  hipGraph_t graph = nullptr;
  hipGraphExec_t exec = nullptr;
  hipEvent_t ev = nullptr;
  ~GraphState() {
    if (exec) (void)hipGraphExecDestroy(exec);
    if (graph) (void)hipGraphDestroy(graph);
    if (ev) (void)hipEventDestroy(ev);
    if (cs) (void)hipStreamDestroy(cs);
  }
};

}  // namespace
}  // namespace phiq

using namespace phiq;

extern "C" phiq_status phiq_etdrk4(phiq_handle h, const phiq_kron_op* op, double tau, int nsteps, double c1,
                                   double c3, double tol, int use_graph, int form, double* u,
                                   phiq_etd_report* rep, hipStream_t stream) {
  if (!h || !u || nsteps < 0 || form < 0 || form > 1) return PHIQ_ERR_INVALID_ARG;
  PHIQ_TRY(validate_op(op));
  if (!std::isfinite(tau) || !std::isfinite(c1) || !std::isfinite(c3) || !std::isfinite(tol))
    return PHIQ_ERR_NONFINITE;
  if (tau < 0 || !(tol > 0)) return PHIQ_ERR_INVALID_ARG;
  if (rep) std::memset(rep, 0, sizeof(*rep));
  if (nsteps == 0) return PHIQ_OK;
  long long N = 1;
  for (int d = 0; d < op->dim; ++d) N *= op->n[d];

  EtdPlans P;
  phiq_report r0{}, r1{}, r2{}, r3{};
  if (form == 0) PHIQ_TRY(phiq_plan_create(h, op, 0.5 * tau, 0, tol, nullptr, &P.half0, &r0, stream));
  PHIQ_TRY(phiq_plan_create(h, op, 0.5 * tau, 1, tol, nullptr, &P.half1, &r1, stream));
  if (form == 0) PHIQ_TRY(phiq_plan_create(h, op, tau, 0, tol, nullptr, &P.full0, &r2, stream));
  PHIQ_TRY(phiq_plan_create(h, op, tau, 3, tol, nullptr, &P.full3, &r3, stream));
  PHIQ_HIP(hipStreamSynchronize(stream));
  for (phiq_plan p : {P.half0, P.half1, P.full0, P.full3})
    if (p) PHIQ_TRY(plan_settle(p));

  double* mem = nullptr;
  const int nbuf = (form == 0) ? kEtdBufN : kEtdComboBufN;
  if (hipMalloc((void**)&mem, sizeof(double) * nbuf * (size_t)N) != hipSuccess) {
    (void)hipGetLastError();
    return PHIQ_ERR_OOM;
  }
  struct Free {
    double* p;
    ~Free() {
      (void)hipDeviceSynchronize();
      (void)hipFree(p);
    }
  } free_mem{mem};
  EtdBufs B{};
  EtdComboBufs BC{};
  double* q = mem;
  auto take = [&](long long k) {
    double* r = q;
    q += k * N;
    return r;
  };
  if (form == 0) {
    B.in2 = take(3);
    B.e_u = take(1);
    B.p1u = take(2);
    B.a = take(1);
    B.fa = take(1);
    B.p1a = take(2);
    B.mix = take(1);
    B.e_a = take(1);
    B.p1m = take(2);
    B.e_full = take(1);
    B.g = take(12);
  } else {
    for (double** b : {&BC.fu, &BC.fa, &BC.fab, &BC.s, &BC.a, &BC.b, &BC.c, &BC.b1, &BC.b2, &BC.b3, &BC.unew})
      *b = take(1);
  }
  auto step = [&](hipStream_t s) {
    return form == 0 ? etd_step(P, B, u, tau, c1, c3, N, s) : etd_step_combo(P, BC, u, tau, c1, c3, N, s);
  };

  // first step eagerly (it also sizes the handle's workspace for all plans)
  PHIQ_TRY(step(stream));
  int eager = 1, replay = 0;
  size_t nodes = 0;
  const bool graph = use_graph && nsteps > 1 && !plan_profiling(P.full3);
  if (graph) {
    GraphState G;
    PHIQ_HIP(hipStreamCreateWithFlags(&G.cs, hipStreamNonBlocking));
    PHIQ_HIP(hipEventCreateWithFlags(&G.ev, hipEventDisableTiming));
    PHIQ_HIP(hipEventRecord(G.ev, stream));
    PHIQ_HIP(hipStreamWaitEvent(G.cs, G.ev, 0));
    PHIQ_HIP(hipStreamBeginCapture(G.cs, hipStreamCaptureModeThreadLocal));
    const phiq_status sc = step(G.cs);
    const hipError_t ec = hipStreamEndCapture(G.cs, &G.graph);
    if (sc != PHIQ_OK) return sc;
    PHIQ_HIP(ec);
    PHIQ_HIP(hipGraphInstantiate(&G.exec, G.graph, nullptr, nullptr, 0));
    PHIQ_HIP(hipGraphGetNodes(G.graph, nullptr, &nodes));
    for (int s = 1; s < nsteps; ++s) {
      PHIQ_HIP(hipGraphLaunch(G.exec, G.cs));
      ++replay;
    }
    PHIQ_HIP(hipEventRecord(G.ev, G.cs));
    PHIQ_HIP(hipStreamWaitEvent(stream, G.ev, 0));
    PHIQ_HIP(hipStreamSynchronize(G.cs));
  } else {
    for (int s = 1; s < nsteps; ++s) {
      PHIQ_TRY(step(stream));
      ++eager;
    }
  }
  PHIQ_HIP(hipStreamSynchronize(stream));
  if (rep) {
    rep->steps_eager = eager;
    rep->steps_graph = replay;
    rep->graph_nodes = (int)nodes;
    rep->l_half = r1.l;
    rep->m_half = r1.m;
    rep->l_full = r3.l;
    rep->m_full = r3.m;
    // form 0: 2 phi_0 at h/2, 3 phi_0..1 at h/2, 1 phi_0 at h, 3 x phi_0..3 at h;
    // form 1: three combinations at h/2 (p = 1) and one at h (p = 3)
    rep->ttm_chains_per_step = (form == 0) ? 2 + 3 * (r1.m + r1.l + 1) + 1 + 3 * (r3.m + 3 * r3.l + 1)
                                           : 3 * combo_chains(1, r1.m, r1.l) + combo_chains(3, r3.m, r3.l);
  }
  return PHIQ_OK;
}
