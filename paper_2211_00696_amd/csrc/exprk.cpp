// phiq_exprk: the exponential Runge-Kutta methods of Section 5 (Table RK:
// exponential Euler, RK2 with c_2, RK3 with c_2 and c_3 = 2/3) on Problem 3.
//
// The paper writes each stage as u + tau sum_j a_ij(-tau A)(g_j - A u).
// With z phi_1(z) = e^z - 1 the terms with A u fold into e^{-c tau A} u,
// so every stage is a sum of phi-actions of u and of source vectors only:
//   Euler:  u+ = e^{-tau A} u + tau phi_1(-tau A) g_1
//   RK2:    U_2 = e^{-c2 tau A} u + c2 tau phi_1(-c2 tau A) g_1
//           u+ = e^{-tau A} u + tau phi_1(-tau A) ((1 - 1/(2 c2)) g_1 + g_2/(2 c2))
//   RK3:    U_2 as RK2;  U_3 = e^{-c3 tau A} u + (2/3) tau phi_1(-c3 tau A) g_1
//                              + 4/(9 c2) tau phi_2(-c3 tau A)(g_2 - g_1)
//           u+ = e^{-tau A} u + tau phi_1(-tau A) g_1 + (3/2) tau phi_2(-tau A)(g_3 - g_1)
// form 0: the vectors of one stage ([u, g_1, ...]) go through one plan
// execution and the stage is combined from their phi_0..phi_p.
// form 1: every stage is one linear combination sum_j phi_j(Z) b_j
// (phiq_plan_execute_combo) with b_0 = u and the scaled sources as b_1, b_2.
#include <cmath>
#include <cstring>
#include <utility>

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

using namespace phiq;

namespace {

struct Plans {
  phiq_plan p[3] = {nullptr, nullptr, nullptr};
  ~Plans() {
    for (phiq_plan q : p)
      if (q) phiq_plan_destroy(q);
  }
};

}  // namespace

namespace {

// form 1: stages as linear combinations.  Buffers G1, G2 (sources), B1, B2
// (scaled combination vectors), U (stage value), W (next u).
phiq_status exprk_combo(const Plans& P, int method, double c2, int nsteps, double tau, int n, double* u,
                        hipStream_t st) {
  const long long N = (long long)n * n;
  const double c3 = 2.0 / 3.0;
  double* mem = nullptr;
  if (hipMalloc((void**)&mem, sizeof(double) * 6 * (size_t)N) != hipSuccess) {
    (void)hipGetLastError();
    return PHIQ_ERR_OOM;
  }
  struct Free {
    double* p;
    ~Free() {
      (void)hipDeviceSynchronize();
      (void)hipFree(p);
    }
  } fr{mem};
  double* G1 = mem;
  double* G2 = mem + N;
  double* B1 = mem + 2 * N;
  double* B2 = mem + 3 * N;
  double* U = mem + 4 * N;
  double* cur = u;
  double* nxt = mem + 5 * N;
  for (int s = 0; s < nsteps; ++s) {
    const double t = s * tau;
    PHIQ_HIP(launch_exprk_stage(cur, nullptr, 0.0, nullptr, 0.0, n, t, G1, nullptr, st));
    if (method == 1) {  // u+ = e^{-tau A} u + phi_1(-tau A) tau g_1
      PHIQ_HIP(launch_exprk_axpby(G1, tau, nullptr, 0.0, B1, N, st));
      const double* b[2] = {cur, B1};
      PHIQ_TRY(phiq_plan_execute_combo(P.p[2], b, nxt, st));
      std::swap(cur, nxt);
      continue;
    }
    {  // U_2 = e^{-c2 tau A} u + phi_1(-c2 tau A) c2 tau g_1
      PHIQ_HIP(launch_exprk_axpby(G1, c2 * tau, nullptr, 0.0, B1, N, st));
      const double* b[2] = {cur, B1};
      PHIQ_TRY(phiq_plan_execute_combo(P.p[0], b, U, st));
    }
    PHIQ_HIP(launch_exprk_stage(U, nullptr, 0.0, nullptr, 0.0, n, t + c2 * tau, G2, nullptr, st));
    if (method == 2) {  // b_1 = tau ((1 - 1/(2 c2)) g_1 + g_2/(2 c2))
      const double b2 = 1.0 / (2.0 * c2);
      PHIQ_HIP(launch_exprk_axpby(G1, tau * (1.0 - b2), G2, tau * b2, B1, N, st));
      const double* b[2] = {cur, B1};
      PHIQ_TRY(phiq_plan_execute_combo(P.p[2], b, nxt, st));
      std::swap(cur, nxt);
      continue;
    }
    {  // U_3 = e^{-c3 tau A} u + phi_1 (2/3) tau g_1 + phi_2 4/(9 c2) tau (g_2 - g_1), at -c3 tau A
      const double w = 4.0 / (9.0 * c2) * tau;
      PHIQ_HIP(launch_exprk_axpby(G1, (2.0 / 3.0) * tau, nullptr, 0.0, B1, N, st));
      PHIQ_HIP(launch_exprk_axpby(G2, w, G1, -w, B2, N, st));
      const double* b[3] = {cur, B1, B2};
      PHIQ_TRY(phiq_plan_execute_combo(P.p[1], b, U, st));
    }
    PHIQ_HIP(launch_exprk_stage(U, nullptr, 0.0, nullptr, 0.0, n, t + c3 * tau, G2, nullptr, st));  // g_3
    {  // u+ = e^{-tau A} u + phi_1 tau g_1 + phi_2 (3/2) tau (g_3 - g_1)
      PHIQ_HIP(launch_exprk_axpby(G1, tau, nullptr, 0.0, B1, N, st));
      PHIQ_HIP(launch_exprk_axpby(G2, 1.5 * tau, G1, -1.5 * tau, B2, N, st));
      const double* b[3] = {cur, B1, B2};
      PHIQ_TRY(phiq_plan_execute_combo(P.p[2], b, nxt, st));
      std::swap(cur, nxt);
    }
  }
  if (cur != u) PHIQ_HIP(launch_exprk_axpby(cur, 1.0, nullptr, 0.0, u, N, st));
  PHIQ_HIP(hipStreamSynchronize(st));
  return PHIQ_OK;
}

}  // namespace

extern "C" phiq_status phiq_exprk(phiq_handle h, const phiq_kron_op* op, int method, double c2, int nsteps, double T,
                                  double tol, const phiq_options* opt, int form, double* u, phiq_report* rep,
                                  hipStream_t st) {
  if (!h || !u || nsteps < 1 || method < 1 || method > 3 || form < 0 || form > 1) return PHIQ_ERR_INVALID_ARG;
  PHIQ_TRY(validate_op(op));
  if (op->dim != 2 || op->n[0] != op->n[1]) return PHIQ_ERR_UNSUPPORTED;  // the source lives on the unit square
  if (!std::isfinite(c2) || !std::isfinite(T) || !std::isfinite(tol)) return PHIQ_ERR_NONFINITE;
  if (!(T > 0) || !(tol > 0) || (method > 1 && !(c2 > 0 && c2 <= 1))) return PHIQ_ERR_INVALID_ARG;
  if (form == 1 && opt && opt->precision == PHIQ_PREC_INT8)
    return PHIQ_ERR_UNSUPPORTED;  // linear combinations: not with the int8-digit form
  const int n = op->n[0];
  const long long N = (long long)n * n;
  const double tau = T / nsteps, c3 = 2.0 / 3.0;
  if (rep) std::memset(rep, 0, sizeof(*rep));

  // plans: [0] at c2 tau (p = 1), [1] at c3 tau (p = 2), [2] at tau (p = method == 3 ? 2 : 1)
  Plans P;
  phiq_report r{};
  const int pfull = (method == 3) ? 2 : 1;
  if (method >= 2) PHIQ_TRY(phiq_plan_create(h, op, c2 * tau, 1, tol, opt, &P.p[0], &r, st));
  if (method == 3) PHIQ_TRY(phiq_plan_create(h, op, c3 * tau, 2, tol, opt, &P.p[1], &r, st));
  PHIQ_TRY(phiq_plan_create(h, op, tau, pfull, tol, opt, &P.p[2], &r, st));
  if (form == 1) {
    PHIQ_TRY(exprk_combo(P, method, c2, nsteps, tau, n, u, st));
    if (rep) *rep = r;
    return PHIQ_OK;
  }

  // R: the stage's vectors [u, g_1, w] (3 N); O: their phi_0..phi_2 (9 N); G2: g_2
  double* mem = nullptr;
  if (hipMalloc((void**)&mem, sizeof(double) * 13 * (size_t)N) != hipSuccess) {
    (void)hipGetLastError();
    return PHIQ_ERR_OOM;
  }
  struct Free {
    double* p;
    ~Free() {
      (void)hipDeviceSynchronize();
      (void)hipFree(p);
    }
  } fr{mem};
  double* R = mem;
  double* O = mem + 3 * N;
  double* G2 = mem + 12 * N;
  auto o = [&](int p, int rr, int k) { return O + ((long long)rr * (p + 1) + k) * N; };

  for (int s = 0; s < nsteps; ++s) {
    const double t = s * tau;
    // R[0] = u, R[1] = g_1
    PHIQ_HIP(launch_exprk_stage(u, nullptr, 0.0, nullptr, 0.0, n, t, R + N, R, st));
    if (method == 1) {
      PHIQ_TRY(phiq_plan_execute(P.p[2], R, 2, O, nullptr, st));
      PHIQ_HIP(launch_exprk_comb(o(1, 0, 0), o(1, 1, 1), tau, nullptr, 0.0, u, N, st));
      continue;
    }
    // U_2 and g_2
    PHIQ_TRY(phiq_plan_execute(P.p[0], R, 2, O, nullptr, st));
    PHIQ_HIP(launch_exprk_stage(o(1, 0, 0), o(1, 1, 1), c2 * tau, nullptr, 0.0, n, t + c2 * tau, G2, nullptr, st));
    if (method == 2) {
      // R[1] = (1 - 1/(2 c2)) g_1 + g_2 / (2 c2)
      const double b2 = 1.0 / (2.0 * c2);
      PHIQ_HIP(launch_exprk_comb(G2, R + N, (1.0 - b2) / b2, nullptr, 0.0, R + N, N, st));  // g_2 + (1-b2)/b2 g_1
      PHIQ_TRY(phiq_plan_execute(P.p[2], R, 2, O, nullptr, st));
      PHIQ_HIP(launch_exprk_comb(o(1, 0, 0), o(1, 1, 1), tau * b2, nullptr, 0.0, u, N, st));
      continue;
    }
    // RK3: U_3 and g_3 (R[2] = g_2 - g_1)
    PHIQ_HIP(launch_exprk_comb(G2, R + N, -1.0, nullptr, 0.0, R + 2 * N, N, st));
    PHIQ_TRY(phiq_plan_execute(P.p[1], R, 3, O, nullptr, st));
    PHIQ_HIP(launch_exprk_stage(o(2, 0, 0), o(2, 1, 1), (2.0 / 3.0) * tau, o(2, 2, 2), 4.0 / (9.0 * c2) * tau, n,
                                t + c3 * tau, G2, nullptr, st));
    // R[2] = g_3 - g_1; u+ = e^{-tau A} u + tau phi_1 g_1 + (3/2) tau phi_2 (g_3 - g_1)
    PHIQ_HIP(launch_exprk_comb(G2, R + N, -1.0, nullptr, 0.0, R + 2 * N, N, st));
    PHIQ_TRY(phiq_plan_execute(P.p[2], R, 3, O, nullptr, st));
    PHIQ_HIP(launch_exprk_comb(o(2, 0, 0), o(2, 1, 1), tau, o(2, 2, 2), 1.5 * tau, u, N, st));
  }
  PHIQ_HIP(hipStreamSynchronize(st));
  if (rep) *rep = r;  // the full-step plan (phi_k(-tau A))
  return PHIQ_OK;
}
