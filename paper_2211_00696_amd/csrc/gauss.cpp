// Execution of a plan with the Gauss rule (Algorithm 1 with the scaling and
// modified squaring of Algorithm phiquadmv): Kronecker chains of 1D
// exponentials, the fused node sum, phi_0 and eq. squaring.
#include "engine.h"

namespace phiq {

// Mode products over axes D-1..1 for nb batches (rotated layout); returns the
// input of the final product over axis 0.  X is FP64; the intermediates T0
// and T1 are FP32 when a lower precision is selected.
phiq_status chain_front(const phiq_plan_s* P, const double* X, long long xs, double* const* Ebase, long long const* es,
                        int nb, void* T0, void* T1, hipStream_t st, Front* f, bool beside) {
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
