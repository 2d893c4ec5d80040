#include "engine.h"

namespace phiq {

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

// The node exponentials of level `level` into its table (allocated on first
// use): the Taylor jobs and sigma squarings, and the lower-precision twin.
phiq_status cc_compute_level(phiq_plan P, int lv, hipStream_t st) {
  phiq_handle h = P->h;
  std::vector<double> theta;
  cc_level_nodes(lv, theta);
  const int cnt = P->cc_count[lv];
  const DevBuf& b = P->cc_E[lv];
  size_t fp64_bytes = 0;
  for (int d = 0; d < P->D; ++d) fp64_bytes += align_up((size_t)cnt * P->n[d] * P->n[d] * sizeof(double));
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
  if (twin_prec(P->opt.precision)) {
    const size_t cnt64 = fp64_bytes / sizeof(double);
    char* tb = (char*)b.p + fp64_bytes;
    PHIQ_HIP(launch_convert((const double*)b.p, (long long)cnt64, P->opt.precision, tb, tb + cnt64 * 2, st,
                            h->guard));
  }
  return PHIQ_OK;
}

// Tables of levels 0..level: new levels are allocated and computed; a level
// whose computation was skipped on the device (a speculative level behind a
// guard, after convergence) is computed again.
phiq_status cc_ensure_level(phiq_plan P, int level, hipStream_t st) {
  phiq_handle h = P->h;
  for (int lv = 0; lv < (int)P->cc_E.size() && lv <= level; ++lv)
    if (!P->cc_valid[lv]) {
      PHIQ_TRY(cc_compute_level(P, lv, st));
      P->cc_valid[lv] = 1;
    }
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
    P->cc_valid.push_back(1);
    if (lp) {
      const size_t cnt64 = fp64_bytes / sizeof(double);
      char* tb = (char*)b.p + fp64_bytes;
      P->twins.t.push_back({(const double*)b.p, cnt64, tb, tb + cnt64 * 2});
    }
    PHIQ_TRY(cc_compute_level(P, lv, st));
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
    h->guard = guard;
    const phiq_status se = cc_ensure_level(P, level, st);
    h->guard = nullptr;
    PHIQ_TRY(se);
    if (guard) P->cc_valid[level] = 0;  // valid only once the host learns the level ran
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
    const size_t rec0 = h->prof.recs.size();
    if (level < cap) PHIQ_TRY(run_level(level + 1, &ctl[level].stop));
    const size_t rec1 = h->prof.recs.size();
    PHIQ_HIP(hipEventSynchronize(h->cc_ev[level]));
    err = h->cc_ctl_host[level].err;
    if (h->cc_ctl_host[level].stop) {
      // the speculative level's launches returned at once: drop their
      // profile records, which would count work that did not run
      h->prof.recs.erase(h->prof.recs.begin() + (long)rec0, h->prof.recs.begin() + (long)rec1);
      converged = true;
      break;
    }
    // level + 1 ran: its table is valid
    if (level < cap) P->cc_valid[level + 1] = 1;
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

}  // namespace phiq
