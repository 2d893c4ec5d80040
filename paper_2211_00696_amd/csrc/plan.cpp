// Plans: norm bound and parameter selection (eq. infnorm_upper_bnd,
// Algorithm setup_quadrature), device layout, and the 1D exponentials of
// the quadrature nodes and the scaling chain (Section 3.3).
#include "engine.h"

namespace phiq {

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
      if (opt.selector != PHIQ_SEL_PAPER && mlp && opt.rule == PHIQ_RULE_GAUSS && opt.m <= 0 && alpha > 1e-12 &&
          l >= 0 && nq >= 0) {
        int lm = l, nm = nq, used = 0;
        const bool ok = (opt.selector == PHIQ_SEL_MLP_EMPIRICAL)
                            ? mlp_choose_empirical(mlp, op, norms, t, p, tol, alpha, l, nq, &lm, &nm, &used)
                            : mlp_choose(mlp, op, norms, t, p, tol, std::pow(10.0, opt.selector_slack), alpha, l,
                                         nq, &lm, &nm, &used);
        if (ok) {
          l = lm;
          nq = nm;
        }
        pp->selector = used;
      }
      if (opt.m > 0 && opt.rule == PHIQ_RULE_GAUSS) nq = opt.m - 1;
      if (opt.rule == PHIQ_RULE_CC && opt.cc_scaling == PHIQ_CC_SCALING_REALIZED && l >= 0 && alpha > 1e-12) {
        l = cc_scaling(tol, p, alpha, opt.c1, opt.c2, op->dim, opt.cc_max_doublings, l);
        nq = quadnodes(tol, p, std::ldexp(alpha, -l), 1.0, PHIQ_RULE_CC);
      }
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

phiq_status plan_build(phiq_handle h, const phiq_kron_op* op, double t, int p, double tol, const phiq_options* uopt,
                       bool transient, phiq_plan* out, phiq_report* rep, hipStream_t st, bool defer_device) {
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
      opt.selector_slack > 12.0 || opt.rhs_per_launch < 0 || opt.selector < PHIQ_SEL_PAPER ||
      opt.selector > PHIQ_SEL_MLP_EMPIRICAL || opt.cc_scaling < PHIQ_CC_SCALING_REALIZED ||
      opt.cc_scaling > PHIQ_CC_SCALING_PAPER)
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
  const bool combo_tab = opt.rule == PHIQ_RULE_GAUSS && p >= 1 && p <= 4;
  const size_t coefc_bytes = combo_tab ? sizeof(double) * (size_t)p * p * P->m : 0;
  const size_t offCoefC = combo_tab ? L.take(coefc_bytes) : 0;
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
  P->coefc = combo_tab ? (double*)(base + offCoefC) : nullptr;
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
  if (combo_tab) {
    const int ld = p * P->m;
    double* hcc = (double*)(hp + offCoefC);
    std::fill(hcc, hcc + (size_t)p * ld, 0.0);
    for (int q = 0; q < p; ++q)
      for (int j = 1; j <= p; ++j) {
        const int k = q - (p - j);
        if (k < 0) continue;
        for (int i = 0; i < P->m; ++i)
          hcc[(size_t)q * ld + (size_t)(p - j) * P->m + i] = std::ldexp(hc[(size_t)k * P->ldcoef + i], l * (p - j));
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

}  // namespace phiq
