#include "engine.h"

namespace phiq {

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

}  // namespace phiq
