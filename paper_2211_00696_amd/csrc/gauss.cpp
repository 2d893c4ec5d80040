// Execution of a plan with the Gauss rule (Algorithm 1 with the scaling and
// modified squaring of Algorithm phiquadmv): Kronecker chains of 1D
// exponentials, the fused node sum, phi_0 and eq. squaring.
#include "engine.h"

namespace phiq {

// Mode products over axes D-1..1 for nb batches (rotated layout); returns the
// input of the final product over axis 0.  X is FP64; the intermediates T0
// and T1 are FP32 when a lower precision is selected.  group > 0 (FP64
// only): the node chains of nb / group vectors at stride xs; batch b takes
// factor b % group in every product, and input b / group in the first
// (later products read their own batch b of the intermediates).
phiq_status chain_front(const phiq_plan_s* P, const double* X, long long xs, double* const* Ebase, long long const* es,
                        int nb, void* T0, void* T1, hipStream_t st, Front* f, bool beside, int group,
                        const TtmSegs* segs) {
  if (group > 0 && (P->opt.precision != PHIQ_PREC_FP64 || nb % group != 0)) return PHIQ_ERR_INVALID_ARG;
  // segs (FP64 only): the batch in segments (TtmSegs), the inputs named there
  if (segs && (P->opt.precision != PHIQ_PREC_FP64 || segs->n < 1 || segs->n > kSegMax || segs->sb[segs->n] != nb))
    return PHIQ_ERR_INVALID_ARG;
  // 1: single-vector chains only (with a batch the per-axis kernels keep more
  // waves per CU busy and were faster at n = 128), and not beside other work
  // on a side stream, where a block that takes a whole CU's LDS waits for a
  // free CU
  const int sp = P->opt.slab_products;
  if (P->D == 3 && P->n[1] == kSlabN && P->n[2] == kSlabN && P->opt.precision == PHIQ_PREC_FP64 && !P->h->guard &&
      group == 0 && !segs && (sp == 2 || (sp == 1 && nb == 1 && !beside))) {
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
    if (group > 0) {
      a.emod = group;
      if (s == 0) a.xdiv = group;
    }
    if (segs) {
      a.seg = *segs;
      if (s > 0)  // later products read their own batch of the intermediates
        for (int q = 0; q < kSegMax; ++q) a.seg.sx[q] = nullptr;
    }
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
                       bool side) {
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

// Device bytes of the intermediate tensors of one Gauss-rule execution on
// g vectors at once: two node batches (max(m + 1, p) tensors per vector)
// and two p-vector squaring iterates per vector.
size_t gauss_ws_bytes(const phiq_plan_s* P, int g) {
  const long long N = P->N;
  const int nb = std::max(P->m + 1, P->p);
  const size_t tbytes = (P->D > 1 ? (size_t)g * nb * N * tensor_elem(P) : 0);
  const size_t ybytes = (size_t)g * P->p * N * sizeof(double);
  return 2 * align_up(tbytes) + 2 * align_up(ybytes);
}

// How many right-hand sides of one phiq_plan_execute share each launch:
// FP64 Gauss plans over at least two axes without slab products; as many as
// the option allows whose intermediates fit in PHIQ_RHS_GROUP_BYTES (and in
// the handle's cap, when one is set).
int rhs_group(const phiq_plan_s* P, int nrhs) {
  if (nrhs < 2 || P->opt.precision != PHIQ_PREC_FP64 || P->opt.rule != PHIQ_RULE_GAUSS || P->p == 0 ||
      P->D < 2 || P->opt.slab_products != 0 || P->opt.rhs_per_launch == 1)
    return 1;
  int g = P->opt.rhs_per_launch > 1 ? std::min(nrhs, P->opt.rhs_per_launch) : nrhs;
  size_t budget = PHIQ_RHS_GROUP_BYTES;
  if (P->h->cap_bytes) budget = std::min(budget, P->h->cap_bytes / 2);
  const size_t per = gauss_ws_bytes(P, 1);
  g = (int)std::min<size_t>((size_t)g, std::max<size_t>(1, budget / std::max<size_t>(per, 1)));
  return g;
}

// The Gauss-rule execution for g vectors (v: g x N, out: g x (p+1) x N) with
// one launch per step for all of them: the first product of the node chains
// takes the pair (vector r, node i) as batch r (m+1) + i, the later products
// are plain batches over the contiguous intermediates, and the node sum, the
// phi_0 product and the squaring products run the g problems side by side
// (TtmArgs::nouter).  Each output element is formed by the same sums in the
// same order as for one vector, so the results are bitwise those of g
// separate executions whenever the same kernels are chosen (the choice can
// depend on a launch's size; at n = 256 the resident-factor kernel sums k in
// another order).
phiq_status execute_gauss_group(phiq_plan P, const double* v, int g, double* out, hipStream_t st) {
  phiq_handle h = P->h;
  const long long N = P->N;
  const int p = P->p, m = P->m;
  if (g < 1 || p < 1 || P->D < 2 || P->opt.precision != PHIQ_PREC_FP64) return PHIQ_ERR_INVALID_ARG;
  const int nb = std::max(m + 1, p);
  const size_t tbytes = (size_t)g * nb * N * sizeof(double);
  const size_t ybytes = (size_t)g * p * N * sizeof(double);
  PHIQ_TRY(ensure(h, h->ws, std::max<size_t>(gauss_ws_bytes(P, g), kAlign)));
  char* wb = (char*)h->ws.p;
  void* T0 = wb;
  void* T1 = wb + align_up(tbytes);
  double* Ya = (double*)(wb + 2 * align_up(tbytes));
  double* Yb = (double*)(wb + 2 * align_up(tbytes) + align_up(ybytes));
  const long long os = (long long)(p + 1) * N;  // one vector's outputs

  double* E[PHIQ_MAX_DIM];
  long long es[PHIQ_MAX_DIM];
  for (int d = 0; d < P->D; ++d) {
    E[d] = P->Enode[d];
    es[d] = (long long)P->n[d] * P->n[d];
  }
  PHIQ_TRY(wait_join(P, st));
  Front f;
  PHIQ_TRY(chain_front(P, v, N, E, es, g * (m + 1), T0, T1, st, &f, false, m + 1));
  const bool direct = (P->l == 0);
  for (int j0 = 0; j0 < p; j0 += 4) {
    TtmArgs a = final_args(P, P->Enode[0], es[0], f, m);
    a.nouter = g;
    a.xo = (long long)(m + 1) * f.xs;
    a.coef = P->coef + (size_t)j0 * P->ldcoef;
    a.ldcoef = P->ldcoef;
    a.np = std::min(4, p - j0);
    a.Y = (direct ? out + N : Ya) + (size_t)j0 * N;
    a.ys = N;
    a.yo = direct ? os : (long long)p * N;
    PHIQ_TRY(L_ttm(h, K_TTM_ACCUM, a, P->opt.precision, st, &P->twins));
  }
  {  // phi_0: slot m of every vector's node batch, one plain batch over g
    Front f0 = f;
    f0.X = elem_offset(f.X, (long long)m * f.xs, f.f32);
    TtmArgs a = final_args(P, P->Ephi0[0], 0, f0, g);
    a.xs = (long long)(m + 1) * f.xs;
    a.O = out;
    a.os = os;
    PHIQ_TRY(L_ttm(h, K_TTM_STORE, a, P->opt.precision, st, &P->twins));
  }
  if (direct) return PHIQ_OK;
  double* cur = Ya;
  for (int k = 0; k < P->l; ++k) {
    double* Ek[PHIQ_MAX_DIM];
    long long e0[PHIQ_MAX_DIM];
    for (int d = 0; d < P->D; ++d) {
      Ek[d] = P->Esq[d] + (size_t)k * P->n[d] * P->n[d];
      e0[d] = 0;
    }
    Front fs;
    PHIQ_TRY(chain_front(P, cur, N, Ek, e0, g * p, T0, T1, st, &fs));
    const bool last = (k == P->l - 1);
    double* dst = last ? out + N : (cur == Ya ? Yb : Ya);
    TtmArgs a = final_args(P, Ek[0], 0, fs, p);
    a.nouter = g;
    a.xo = (long long)p * fs.xs;
    a.O = dst;
    a.os = N;
    a.oo = last ? os : (long long)p * N;
    a.Yprev = cur;
    a.yps = N;
    a.ypo = (long long)p * N;
    PHIQ_TRY(L_ttm(h, K_TTM_SQUARE, a, P->opt.precision, st, &P->twins));
    cur = dst;
  }
  return PHIQ_OK;
}

// ws (nullable): a caller-provided workspace of ws_cap bytes used instead of
// the handle's (no allocation; PHIQ_ERR_OOM when it is too small).
phiq_status execute_gauss(phiq_plan P, const double* v, double* out, hipStream_t st, void* ws,
                          size_t ws_cap) {
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

}  // namespace phiq
