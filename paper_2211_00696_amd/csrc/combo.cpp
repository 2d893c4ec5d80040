#include "engine.h"

namespace phiq {

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
// FP64 with every b_1..b_p set (p <= 4): one batch per mode product for the
// node chains of all b_j and phi_0's chain of b_0 (batch segments), then one
// node sum for all of them with the plan's combined coefficients.
phiq_status execute_combo_fused(phiq_plan P, const double* const* b, double* out, hipStream_t st) {
  phiq_handle h = P->h;
  const long long N = P->N;
  const int p = P->p, m = P->m;
  TtmSegs sg{};
  int nb = 0;
  for (int j = p; j >= 1; --j) {
    sg.sb[sg.n] = nb;
    sg.se[sg.n] = 0;
    sg.sx[sg.n] = b[j];
    ++sg.n;
    nb += m;
  }
  const bool have0 = b[0] != nullptr;
  if (have0) {  // slot m of the node tables is phi_0's factor
    sg.sb[sg.n] = nb;
    sg.se[sg.n] = m;
    sg.sx[sg.n] = b[0];
    ++sg.n;
    nb += 1;
  }
  sg.sb[sg.n] = nb;
  const size_t tbytes = (size_t)std::max(nb, p) * N * sizeof(double);
  const size_t ybytes = (size_t)p * N * sizeof(double);
  PHIQ_TRY(ensure(h, h->ws, 2 * align_up(tbytes) + 2 * align_up(ybytes)));
  char* wb = (char*)h->ws.p;
  void* T0 = wb;
  void* T1 = wb + align_up(tbytes);
  double* Ya = (double*)(wb + 2 * align_up(tbytes));
  double* Yb = (double*)(wb + 2 * align_up(tbytes) + align_up(ybytes));

  double* E[PHIQ_MAX_DIM];
  long long es[PHIQ_MAX_DIM];
  for (int d = 0; d < P->D; ++d) {
    E[d] = P->Enode[d];
    es[d] = (long long)P->n[d] * P->n[d];
  }
  PHIQ_TRY(wait_join(P, st));
  Front f;
  PHIQ_TRY(chain_front(P, nullptr, 0, E, es, nb, T0, T1, st, &f, false, 0, &sg));
  if (have0) {  // phi_0 b_0 into out: the last product of the b_0 segment
    Front f0 = f;
    f0.X = elem_offset(f.X, (long long)p * m * f.xs, f.f32);
    TtmArgs a = final_args(P, P->Ephi0[0], 0, f0, 1);
    a.O = out;
    a.os = 0;
    PHIQ_TRY(L_ttm(h, K_TTM_STORE, a, P->opt.precision, st, &P->twins));
  }
  // node sum of all b_j: y_q = sum over (j, i) of the combined coefficients;
  // without squaring only y_p, added to phi_0 b_0 in out
  const bool direct = (P->l == 0);
  TtmArgs a = final_args(P, P->Enode[0], es[0], f, p * m);
  a.emod = m;
  a.ldcoef = p * m;
  a.coef = P->coefc + (direct ? (size_t)(p - 1) * a.ldcoef : 0);
  a.np = direct ? 1 : p;
  a.Y = direct ? out : Ya;
  a.ys = N;
  a.yacc = (direct && have0) ? 1 : 0;
  PHIQ_TRY(L_ttm(h, K_TTM_ACCUM, a, P->opt.precision, st, &P->twins));
  if (direct) return PHIQ_OK;
  return combo_squaring(P, Ya, Yb, p, out, have0, false, T0, T1, st);
}

phiq_status execute_combo(phiq_plan P, const double* const* b, double* out, hipStream_t st) {
  phiq_handle h = P->h;
  const long long N = P->N;
  int pe = 0;  // highest order with a vector
  bool all = true;
  for (int j = 1; j <= P->p; ++j) {
    if (b[j]) pe = j;
    all = all && b[j];
  }
  if (all && P->coefc && P->opt.precision == PHIQ_PREC_FP64 && P->opt.slab_products == 0 && P->D >= 2 &&
      P->opt.rhs_per_launch != 1)
    return execute_combo_fused(P, b, out, st);
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

}  // namespace phiq
