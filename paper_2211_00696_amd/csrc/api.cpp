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
#include "engine.h"

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
  const int grp = rhs_group(plan, nrhs);
  for (int r = 0; r < nrhs;) {
    const double* vr = v + (size_t)r * N;
    double* outr = out + (size_t)r * (plan->p + 1) * N;
    const int gr = std::min(grp, nrhs - r);
    r += gr;
    if (gr > 1) {
      PHIQ_TRY(execute_gauss_group(plan, vr, gr, outr, stream));
    } else if (plan->opt.precision == PHIQ_PREC_INT8) {
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
