// phiq_action_batched: many independent phi-actions in one persistent launch.
//
// The host turns every problem of the batch into stages (Algorithm 6 per
// problem with Algorithm 1's quadrature and the modified squaring):
//   1D exponentials  powers Z^2..Z^K by doubling rounds, Taylor sums for all
//                    node coefficients, sigma_d squarings, the scaling chain
//                    E^(k) = E^(k-1)^2 (k = 1..l, E^(l) = the phi_0 factor);
//   per vector       node chunks (<= 4 nodes): D-1 mode products, then the
//                    last mode product with the node sum fused; l squaring
//                    steps: D-1 mode products over the p orders, then the
//                    last one with the squaring combination fused; phi_0.
// Each stage belongs to one dependency group (the stages of a step whose
// results are consumed together) and reads the results of at most two
// groups.  Stages are ordered by their depth in this dependency graph
// (largest first within a depth); one launch runs each depth.
#include <algorithm>
#include <cmath>
#include <cstdint>
#include <cstring>
#include <numeric>
#include <vector>

#include <hip/hip_runtime_api.h>

#include "phiq_internal.h"

#define PHIQ_TRY(x)                  \
  do {                               \
    const phiq_status s_ = (x);      \
    if (s_ != PHIQ_OK) return s_;    \
  } while (0)
#define PHIQ_HIP(x)                                  \
  do {                                               \
    if ((x) != hipSuccess) {                         \
      (void)hipGetLastError();                       \
      return PHIQ_ERR_HIP;                           \
    }                                                \
  } while (0)

namespace phiq {
namespace {

constexpr size_t kAl = 256;
inline size_t al(size_t x) { return (x + kAl - 1) / kAl * kAl; }
inline long long cdiv(long long a, long long b) { return (a + b - 1) / b; }
constexpr int kChunk = 4;  // nodes per quadrature chunk (node-sum epilogue width)
constexpr long long kBatchGrid = 2048;  // workgroups per launch at most (multiple of 8)
// polls of one dependency wait in the persistent launch before it gives up
// (each poll sleeps 256 cycles: several seconds in all, far beyond any tile)
constexpr long long kPersistSpinLimit = 1ll << 23;

struct Prob {
  const phiq_problem* pr = nullptr;
  PlanParams pp{};
  int D = 0;
  int n[PHIQ_MAX_DIM] = {};
  long long N = 1;
  std::vector<double> theta, w;
  size_t base = 0;  // problem region offset
  size_t zp[PHIQ_MAX_DIM] = {}, enode[PHIQ_MAX_DIM] = {}, esq[PHIQ_MAX_DIM] = {}, ephi0[PHIQ_MAX_DIM] = {},
         s0[PHIQ_MAX_DIM] = {}, s1[PHIQ_MAX_DIM] = {};
  size_t ws = 0;     // first vector's workspace; vector r at ws + r * rhs_bytes
  size_t t_elems = 0, y_elems = 0, rhs_bytes = 0, bytes = 0;
  size_t z1[PHIQ_MAX_DIM] = {}, coef = 0;  // inside the upload region
};

struct Graph {
  std::vector<BatchStage> st;
  std::vector<int> lvl;
  std::vector<int> glevel, gneed;
  std::vector<BatchTaylor> tj;
  int group() {
    glevel.push_back(-1);
    gneed.push_back(0);
    return (int)glevel.size() - 1;
  }
  void add(BatchStage s, int signal, int w0 = -1, int w1 = -1) {
    int L = 0;
    if (w0 >= 0) L = std::max(L, glevel[w0] + 1);
    if (w1 >= 0) L = std::max(L, glevel[w1] + 1);
    s.signal = signal;
    s.wait0 = w0;
    s.wait1 = w1;
    glevel[signal] = std::max(glevel[signal], L);
    gneed[signal] += s.ntiles;
    st.push_back(s);
    lvl.push_back(L);
  }
};

inline bool aligned16(const void* p) { return ((uintptr_t)p & 15u) == 0; }

BatchStage gemm(const double* A, const double* B, double* C, int n) {
  BatchStage s{};
  s.type = kStageGemm;
  s.M = s.K = s.L = n;
  s.E = A;
  s.X = B;
  s.O = C;
  s.ntiles = (int)(cdiv(n, kBatchTile) * cdiv(n, kBatchTile));
  return s;
}

BatchStage ttm(int type, const double* E, long long es, const double* X, long long xs, int n, long long N, int nb) {
  BatchStage s{};
  s.type = type;
  s.M = s.K = n;
  s.L = (int)(N / n);
  s.nb = nb;
  s.E = E;
  s.es = es;
  s.X = X;
  s.xs = xs;
  s.vec = (n % 2 == 0) && aligned16(E) && aligned16(X) && es % 2 == 0 && xs % 2 == 0;
  // the single-problem kernels' fastest shapes at n >= 128: 64 x 128 stores,
  // eight-wave node sums and squaring steps (the thresholds from batch timings)
  if (type == kStageStore && n >= kBatchWideM) {
    s.type = kStageStoreWide;
    s.ntiles = (int)(cdiv(s.M, kBatchTile) * cdiv(s.L, kBatchWideN) * nb);
    return s;
  }
  if (n >= kBatchWaves8M && type == kStageAccum) s.type = kStageAccumWide;
  if (n >= kBatchWaves8M && type == kStageSquare) s.type = kStageSquareWide;
  const long long per = cdiv(s.M, kBatchTile) * cdiv(s.L, kBatchTile);
  s.ntiles = (int)(type == kStageStore ? per * nb : per);
  return s;
}

// Stages of problem P with device pointers relative to `base` (the arena)
// and `up` (the upload region inside it).
void build_problem(const Prob& P, char* base, char* up, Graph& g) {
  const phiq_problem& pr = *P.pr;
  const int D = P.D, p = pr.p, l = P.pp.l, m = P.pp.m, K = P.pp.K;
  const long long N = P.N;
  char* pb = base + P.base;
  auto dp = [&](size_t off) { return (double*)(pb + off); };
  const double* Z1[PHIQ_MAX_DIM];
  double *Zp[PHIQ_MAX_DIM], *Enode[PHIQ_MAX_DIM], *Esq[PHIQ_MAX_DIM], *Ephi0[PHIQ_MAX_DIM], *S[2][PHIQ_MAX_DIM];
  for (int d = 0; d < D; ++d) {
    Z1[d] = (const double*)(up + P.z1[d]);
    Zp[d] = dp(P.zp[d]);
    Enode[d] = dp(P.enode[d]);
    Esq[d] = dp(P.esq[d]);
    Ephi0[d] = dp(P.ephi0[d]);
    S[0][d] = dp(P.s0[d]);
    S[1][d] = dp(P.s1[d]);
  }
  auto zpow = [&](int d, int j) -> const double* {
    return j == 1 ? Z1[d] : Zp[d] + (size_t)(j - 2) * P.n[d] * P.n[d];
  };

  // ---- 1D exponentials ----
  const int gfac = g.group();  // every final node / E^(0) factor written
  for (int d = 0; d < D; ++d) {
    const int n = P.n[d];
    const size_t nn = (size_t)n * n;
    int gprev = -1;
    for (int pw = 1; pw < K; pw *= 2) {  // Z^{j+pw} = Z^j Z^pw
      const int gr = g.group();
      for (int j = 1; j <= pw && j + pw <= K; ++j)
        g.add(gemm(zpow(d, j), zpow(d, pw), (double*)zpow(d, j + pw), n), gr, gprev);
      gprev = gr;
    }
    // Taylor targets: Gauss nodes c = 1 - theta_q, then E^(0) (c = 1)
    struct Tg {
      double c;
      double* dst;
      int slot;
    };
    std::vector<Tg> tg;
    for (int q = 0; q < m; ++q) tg.push_back({1.0 - P.theta[q], Enode[d] + q * nn, q});
    tg.push_back({1.0, (l > 0) ? Esq[d] : Ephi0[d], m});
    const int sg = P.pp.sigma[d];
    const int gtay = sg > 0 ? g.group() : gfac;
    for (size_t t0 = 0; t0 < tg.size(); t0 += kTaylorTargets) {
      BatchTaylor jb{};
      jb.Z1 = Z1[d];
      jb.Zp = Zp[d];
      jb.n = n;
      jb.K = K;
      for (size_t t = t0; t < tg.size() && jb.nt < kTaylorTargets; ++t) {
        jb.c[jb.nt] = tg[t].c;
        jb.dst[jb.nt] = sg > 0 ? S[0][d] + (size_t)tg[t].slot * nn : tg[t].dst;
        ++jb.nt;
      }
      BatchStage s{};
      s.type = kStageTaylor;
      s.M = n;
      s.aux = (int)g.tj.size();
      s.ntiles = (int)cdiv((long long)nn, kBatchTaylorChunk);
      g.tj.push_back(jb);
      g.add(s, gtay, gprev);
    }
    int gs = gtay;
    for (int r = 1; r <= sg; ++r) {  // X <- X^2, sigma_d times
      const int gr = (r == sg) ? gfac : g.group();
      for (const auto& t : tg) {
        const double* src = S[(r - 1) % 2][d] + (size_t)t.slot * nn;
        double* dst = (r == sg) ? t.dst : S[r % 2][d] + (size_t)t.slot * nn;
        g.add(gemm(src, src, dst, n), gr, gs);
      }
      gs = gr;
    }
  }
  std::vector<int> gsq(l + 1, gfac);  // gsq[k]: E^(k) of every axis written
  for (int k = 1; k <= l; ++k) {
    gsq[k] = g.group();
    for (int d = 0; d < D; ++d) {
      const size_t nn = (size_t)P.n[d] * P.n[d];
      const double* src = Esq[d] + (k - 1) * nn;
      g.add(gemm(src, src, (k < l) ? Esq[d] + k * nn : Ephi0[d], P.n[d]), gsq[k], gsq[k - 1]);
    }
  }

  // ---- per vector ----
  const double* coef = (const double*)(up + P.coef);
  for (int r = 0; r < pr.nrhs; ++r) {
    const double* v = pr.v + (size_t)r * N;
    double* out = pr.out + (size_t)r * (p + 1) * N;
    char* wsb = pb + P.ws + r * P.rhs_bytes;
    double* T[2] = {(double*)wsb, (double*)(wsb + al(P.t_elems * 8))};
    double* Ya = (double*)(wsb + 2 * al(P.t_elems * 8));
    double* Yb = (double*)(wsb + 2 * al(P.t_elems * 8) + al(P.y_elems * 8));
    int prev = -1;
    auto next = [&](BatchStage s, int extra) {
      const int gg = g.group();
      g.add(s, gg, prev, extra);
      prev = gg;
    };
    // modes D-1..1 (rotated), returns the input of the last mode product
    auto front = [&](double* const* E, long long const* es, const double* X, long long xs, int nb,
                     int first_extra) -> const double* {
      const double* cur = X;
      long long cxs = xs;
      int extra = first_extra;
      for (int s = 0; s + 1 < D; ++s) {
        const int d = D - 1 - s;
        BatchStage st = ttm(kStageStore, E[d], es[d], cur, cxs, P.n[d], N, nb);
        st.O = T[s % 2];
        st.os = N;
        next(st, extra);
        extra = -1;
        cur = T[s % 2];
        cxs = N;
      }
      return cur;
    };
    if (p > 0) {
      double* Y = (l == 0) ? out + N : Ya;
      for (int q0 = 0; q0 < m; q0 += kChunk) {
        const int nq = std::min(kChunk, m - q0);
        double* E[PHIQ_MAX_DIM];
        long long es[PHIQ_MAX_DIM];
        for (int d = 0; d < D; ++d) {
          es[d] = (long long)P.n[d] * P.n[d];
          E[d] = Enode[d] + q0 * es[d];
        }
        const int extra = (q0 == 0) ? gfac : -1;
        const double* X = front(E, es, v, 0, nq, extra);
        BatchStage st = ttm(kStageAccum, E[0], es[0], X, D > 1 ? N : 0, P.n[0], N, nq);
        st.coef = coef + q0;
        st.ldcoef = m;
        st.np = p;
        st.Y = Y;
        st.ys = N;
        st.accumulate = q0 > 0;
        next(st, D > 1 ? -1 : extra);
      }
      double* cur = Ya;
      for (int k = 0; k < l; ++k) {
        double* E[PHIQ_MAX_DIM];
        long long es[PHIQ_MAX_DIM];
        for (int d = 0; d < D; ++d) {
          E[d] = Esq[d] + (size_t)k * P.n[d] * P.n[d];
          es[d] = 0;
        }
        double* dst = (k == l - 1) ? out + N : (cur == Ya ? Yb : Ya);
        const double* X = front(E, es, cur, N, p, gsq[k]);
        BatchStage st = ttm(kStageSquare, E[0], 0, X, N, P.n[0], N, 1);
        st.O = dst;
        st.os = N;
        st.Y = cur;
        st.ys = N;
        st.np = p;
        next(st, D > 1 ? -1 : gsq[k]);
        cur = dst;
      }
    }
    // phi_0 = (exp(-tA^0) (x) ... ) v
    {
      double* E[PHIQ_MAX_DIM];
      long long es[PHIQ_MAX_DIM];
      for (int d = 0; d < D; ++d) {
        E[d] = Ephi0[d];
        es[d] = 0;
      }
      const double* X = front(E, es, v, 0, 1, gsq[l]);
      BatchStage st = ttm(kStageStore, E[0], 0, X, 0, P.n[0], N, 1);
      st.O = out;
      st.os = 0;
      next(st, D > 1 ? -1 : gsq[l]);
    }
  }
}

struct Launch {
  int type, stage_begin, stage_end;
  long long tile_begin, tile_end;
};

struct Built {
  std::vector<BatchStage> st;  // by depth, then type
  std::vector<Launch> launches;
  std::vector<BatchTaylor> tj;
  std::vector<long long> level_tile;  // first tile of each depth, then the total
  std::vector<int> stage_level;
  int ngroups = 0;
  long long total = 0;
};

// Kernel variant of a stage within its type: orders (Accum, Square) and
// 16-byte staging.
int key(const BatchStage& s) {
  const bool acc_sq = s.type == kStageAccum || s.type == kStageSquare || s.type == kStageAccumWide ||
                      s.type == kStageSquareWide;
  const int np = acc_sq ? s.np : 0;
  const int vec = (acc_sq || s.type == kStageStore || s.type == kStageStoreWide) ? s.vec : 0;
  return np * 2 + vec;
}

void build_all(const std::vector<Prob>& probs, char* base, char* up, Built* b, int* depth) {
  Graph g;
  for (const auto& P : probs) build_problem(P, base, up, g);
  std::vector<int> order(g.st.size());
  std::iota(order.begin(), order.end(), 0);
  std::stable_sort(order.begin(), order.end(), [&](int a, int c) {
    if (g.lvl[a] != g.lvl[c]) return g.lvl[a] < g.lvl[c];
    if (g.st[a].type != g.st[c].type) return g.st[a].type < g.st[c].type;
    if (key(g.st[a]) != key(g.st[c])) return key(g.st[a]) < key(g.st[c]);
    return g.st[a].ntiles > g.st[c].ntiles;
  });
  b->st.clear();
  b->st.reserve(order.size());
  b->level_tile.clear();
  b->stage_level.clear();
  long long t = 0;
  for (int i : order) {
    BatchStage s = g.st[i];
    while ((int)b->level_tile.size() <= g.lvl[i]) b->level_tile.push_back(t);
    s.tile0 = t;
    s.need0 = s.wait0 >= 0 ? g.gneed[s.wait0] : 0;
    s.need1 = s.wait1 >= 0 ? g.gneed[s.wait1] : 0;
    t += s.ntiles;
    b->st.push_back(s);
    b->stage_level.push_back(g.lvl[i]);
  }
  b->level_tile.push_back(t);
  b->launches.clear();
  for (size_t i = 0; i < b->st.size(); ++i) {
    const BatchStage& s = b->st[i];
    if (b->launches.empty() || b->launches.back().type != s.type ||
        key(b->st[b->launches.back().stage_begin]) != key(s) ||
        b->stage_level[b->launches.back().stage_begin] != b->stage_level[i])
      b->launches.push_back({s.type, (int)i, (int)i, s.tile0, s.tile0});
    b->launches.back().stage_end = (int)i + 1;
    b->launches.back().tile_end = s.tile0 + s.ntiles;
  }
  b->tj = g.tj;
  b->ngroups = (int)g.glevel.size();
  b->total = t;
  *depth = (int)b->level_tile.size() - 1;
}

bool overlaps(std::vector<std::pair<uintptr_t, uintptr_t>> iv) {
  std::sort(iv.begin(), iv.end());
  for (size_t i = 1; i < iv.size(); ++i)
    if (iv[i].first < iv[i - 1].second) return true;
  return false;
}

// Everything the host decides about a batch: validated problems, which run
// in the persistent launch, and the arena layout.
struct Schedule {
  phiq_options opt{};
  std::vector<Prob> pl;     // persistent launch
  std::vector<int> rest;    // one plan each
  size_t up_off = 0;        // upload region offset in the arena
  size_t up_bytes = 0;      // upload region bytes
  size_t st_off = 0, tj_off = 0;  // inside the upload region
  size_t pc_off = 0;              // persistent launch: tile counter, error flag, group counters (zeroed by the upload)
  size_t total = 0;         // arena bytes
  Built b;
  int depth = 0;

  phiq_status make(int nprob, const phiq_problem* probs, const phiq_options* uopt, const float* mlp) {
    phiq_options_default(&opt);
    if (uopt) opt = *uopt;
    std::vector<std::pair<uintptr_t, uintptr_t>> outs, ins;
    for (int i = 0; i < nprob; ++i) {
      const phiq_problem& pr = probs[i];
      PHIQ_TRY(validate_op(&pr.op));
      if (!std::isfinite(pr.t) || !std::isfinite(pr.tol)) return PHIQ_ERR_NONFINITE;
      if (pr.p < 0 || pr.p > PHIQ_MAX_P || !(pr.tol > 0) || pr.nrhs < 1 || !pr.v || !pr.out)
        return PHIQ_ERR_INVALID_ARG;
      uintptr_t N = 1;
      for (int d = 0; d < pr.op.dim; ++d) N *= (uintptr_t)pr.op.n[d];
      outs.push_back({(uintptr_t)pr.out, (uintptr_t)pr.out + (uintptr_t)pr.nrhs * (pr.p + 1) * N * 8});
      ins.push_back({(uintptr_t)pr.v, (uintptr_t)pr.v + (uintptr_t)pr.nrhs * N * 8});
    }
    // outputs are disjoint; an input may be shared by problems but overlaps no output
    if (overlaps(outs)) return PHIQ_ERR_INVALID_ARG;
    for (const auto& v : ins)
      for (const auto& o : outs)
        if (v.first < o.second && o.first < v.second) return PHIQ_ERR_INVALID_ARG;
    if (opt.rule != PHIQ_RULE_GAUSS && opt.rule != PHIQ_RULE_CC) return PHIQ_ERR_INVALID_ARG;
    const bool persistent_ok = opt.rule == PHIQ_RULE_GAUSS && opt.precision == PHIQ_PREC_FP64;
    for (int i = 0; i < nprob; ++i) {
      const phiq_problem& pr = probs[i];
      if (!persistent_ok || pr.p > 4) {
        rest.push_back(i);
        continue;
      }
      Prob P;
      P.pr = &pr;
      PHIQ_TRY(select_params(&pr.op, pr.t, pr.p, pr.tol, opt, &P.pp, mlp));
      P.D = pr.op.dim;
      for (int d = 0; d < P.D; ++d) {
        P.n[d] = pr.op.n[d];
        P.N *= P.n[d];
      }
      if (P.pp.m > 0) {
        P.theta.resize(P.pp.m);
        P.w.resize(P.pp.m);
        gauss_legendre(P.pp.m, P.theta.data(), P.w.data());
      }
      pl.push_back(std::move(P));
    }
    if (pl.empty()) return PHIQ_OK;
    // problem regions, then the upload region
    size_t off = 0;
    for (auto& P : pl) {
      P.base = off;
      size_t o = 0;
      const int m = P.pp.m, l = P.pp.l, K = P.pp.K;
      for (int d = 0; d < P.D; ++d) {
        const size_t nn = (size_t)P.n[d] * P.n[d] * 8;
        P.zp[d] = o;
        o += al(nn * std::max(0, K - 1));
        P.enode[d] = o;
        o += al(nn * m);
        P.esq[d] = o;
        o += al(nn * std::max(1, l));
        P.ephi0[d] = o;
        o += al(nn);
        P.s0[d] = o;
        if (P.pp.sigma[d] >= 1) o += al(nn * (m + 1));
        P.s1[d] = o;
        if (P.pp.sigma[d] >= 2) o += al(nn * (m + 1));
      }
      P.t_elems = P.D > 1 ? (size_t)std::max(kChunk, P.pr->p) * P.N : 0;
      P.y_elems = (P.pr->p > 0 && l > 0) ? (size_t)P.pr->p * P.N : 0;
      P.rhs_bytes = 2 * al(P.t_elems * 8) + 2 * al(P.y_elems * 8);
      P.ws = o;
      o += P.rhs_bytes * P.pr->nrhs;
      P.bytes = o;
      off += al(o);
    }
    up_off = off;
    size_t uo = 0;
    for (auto& P : pl) {
      for (int d = 0; d < P.D; ++d) {
        P.z1[d] = uo;
        uo += al((size_t)P.n[d] * P.n[d] * 8);
      }
      P.coef = uo;
      uo += al((size_t)std::max(1, P.pr->p) * std::max(1, P.pp.m) * 8);
    }
    build_all(pl, nullptr, nullptr, &b, &depth);  // counts only
    st_off = uo;
    uo += al(b.st.size() * sizeof(BatchStage));
    tj_off = uo;
    uo += al(std::max<size_t>(1, b.tj.size()) * sizeof(BatchTaylor));
    pc_off = uo;
    uo += al(sizeof(BatchPersistCtl)) + al((size_t)std::max(1, b.ngroups) * sizeof(unsigned));
    up_bytes = uo;
    total = up_off + uo;
    return PHIQ_OK;
  }

  // Every address a stage may touch lies in the arena or in its problem's
  // v / out, and every group a stage reads is complete before the launch of
  // the stage's depth starts.  Run before the launches.
  phiq_status check(const char* base) const {
    struct R {
      uintptr_t lo, hi;
    };
    std::vector<R> ok;
    ok.push_back({(uintptr_t)base, (uintptr_t)base + total});
    for (const auto& P : pl) {
      const uintptr_t N = (uintptr_t)P.N;
      ok.push_back({(uintptr_t)P.pr->v, (uintptr_t)P.pr->v + P.pr->nrhs * N * 8});
      ok.push_back({(uintptr_t)P.pr->out, (uintptr_t)P.pr->out + P.pr->nrhs * (P.pr->p + 1) * N * 8});
    }
    auto in = [&](const void* p, long long elems) {
      if (elems <= 0) return true;
      const uintptr_t a = (uintptr_t)p, e = a + (uintptr_t)elems * 8;
      for (const auto& r : ok)
        if (a >= r.lo && e <= r.hi) return true;
      return false;
    };
    std::vector<long long> end(b.ngroups, 0);
    long long t = 0;
    for (const auto& s : b.st) {
      if (s.tile0 != t || s.ntiles < 1) return PHIQ_ERR_INVALID_ARG;
      t += s.ntiles;
      if (s.signal < 0 || s.signal >= b.ngroups) return PHIQ_ERR_INVALID_ARG;
      end[s.signal] = std::max(end[s.signal], s.tile0 + s.ntiles);
    }
    if (t != b.total || b.level_tile.empty() || b.level_tile.back() != t) return PHIQ_ERR_INVALID_ARG;
    for (size_t i = 0; i < b.st.size(); ++i) {
      const BatchStage& s = b.st[i];
      const int lv = b.stage_level[i];
      if (s.tile0 < b.level_tile[lv] || s.tile0 + s.ntiles > b.level_tile[lv + 1]) return PHIQ_ERR_INVALID_ARG;
      for (int w : {s.wait0, s.wait1})
        if (w >= 0 && (w >= b.ngroups || end[w] > b.level_tile[lv])) return PHIQ_ERR_INVALID_ARG;
      const long long MK = (long long)s.M * s.K, LK = (long long)s.L * s.K, ML = (long long)s.M * s.L;
      bool good = true;
      switch (s.type) {
        case kStageGemm:
          good = in(s.E, MK) && in(s.X, MK) && in(s.O, MK);
          break;
        case kStageTaylor: {
          if (s.aux < 0 || s.aux >= (int)b.tj.size()) return PHIQ_ERR_INVALID_ARG;
          const BatchTaylor& j = b.tj[s.aux];
          const long long nn = (long long)j.n * j.n;
          good = j.K >= 1 && j.K <= kMaxTaylorDegree && j.nt >= 1 && j.nt <= kTaylorTargets && in(j.Z1, nn) &&
                 in(j.Zp, nn * (j.K - 1)) && (long long)s.ntiles * kBatchTaylorChunk >= nn;
          for (int q = 0; q < j.nt && good; ++q) good = in(j.dst[q], nn);
          break;
        }
        case kStageStore:
        case kStageStoreWide:
          for (int q = 0; q < s.nb && good; ++q)
            good = in(s.E + q * s.es, MK) && in(s.X + q * s.xs, LK) && in(s.O + q * s.os, ML);
          break;
        case kStageAccum:
        case kStageAccumWide:
          if (s.np < 1 || s.np > 4) return PHIQ_ERR_INVALID_ARG;
          for (int q = 0; q < s.nb && good; ++q) good = in(s.E + q * s.es, MK) && in(s.X + q * s.xs, LK);
          for (int q = 0; q < s.np && good; ++q)
            good = in(s.Y + q * s.ys, ML) && in(s.coef + q * s.ldcoef, s.nb);
          break;
        case kStageSquare:
        case kStageSquareWide:
          if (s.np < 1 || s.np > 4) return PHIQ_ERR_INVALID_ARG;
          good = in(s.E, MK);
          for (int q = 0; q < s.np && good; ++q)
            good = in(s.X + q * s.xs, LK) && in(s.Y + q * s.ys, ML) && in(s.O + q * s.os, ML);
          break;
        default:
          return PHIQ_ERR_INVALID_ARG;
      }
      if (!good) return PHIQ_ERR_INVALID_ARG;
    }
    return PHIQ_OK;
  }
};

}  // namespace
}  // namespace phiq

using namespace phiq;

extern "C" phiq_status phiq_batch_info(int nprob, const phiq_problem* probs, const phiq_options* opt,
                                       phiq_batch_stats* info) {
  if (nprob < 0 || (nprob > 0 && !probs) || !info) return PHIQ_ERR_INVALID_ARG;
  std::memset(info, 0, sizeof(*info));
  Schedule S;
  PHIQ_TRY(S.make(nprob, probs, opt, nullptr));
  info->persistent = (int)S.pl.size();
  info->separate = (int)S.rest.size();
  if (S.pl.empty()) return PHIQ_OK;
  // the same schedule at a stand-in arena address (nothing is dereferenced)
  const char* fake = (const char*)(uintptr_t)((uintptr_t)1 << 44);
  build_all(S.pl, (char*)fake, (char*)fake + S.up_off, &S.b, &S.depth);
  PHIQ_TRY(S.check(fake));
  info->stages = (long long)S.b.st.size();
  info->tiles = S.b.total;
  info->depth = S.depth;
  info->launches = (int)S.b.launches.size();
  info->groups = S.b.ngroups;
  info->arena_bytes = S.total;
  info->upload_bytes = S.up_bytes;
  return PHIQ_OK;
}

extern "C" phiq_status phiq_action_batched(phiq_handle h, int nprob, const phiq_problem* probs,
                                           const phiq_options* uopt, hipStream_t stream) {
  if (!h || nprob < 0 || (nprob > 0 && !probs)) return PHIQ_ERR_INVALID_ARG;
  if (nprob == 0) return PHIQ_OK;
  Schedule S;
  PHIQ_TRY(S.make(nprob, probs, uopt, handle_mlp(h)));
  const phiq_options& opt = S.opt;
  if (!S.pl.empty()) {
    if (opt.workspace_cap && S.total > opt.workspace_cap) return PHIQ_ERR_OOM;
    void* arena = nullptr;
    PHIQ_TRY(batch_arena(h, S.total, &arena));
    char* base = (char*)arena;
    char* up = base + S.up_off;
    build_all(S.pl, base, up, &S.b, &S.depth);
    PHIQ_TRY(S.check(base));
    int slot = 0;
    void* hostp = nullptr;
    PHIQ_TRY(batch_stage(h, S.up_bytes, &slot, &hostp));
    char* hp = (char*)hostp;
    std::memset(hp, 0, S.up_bytes);
    for (auto& P : S.pl) {
      const phiq_problem& pr = *P.pr;
      for (int d = 0; d < P.D; ++d) {
        // Z^1 = -t 2^{-l-sigma_d} A^d
        const double sc = -pr.t * std::ldexp(1.0, -P.pp.l - P.pp.sigma[d]);
        double* z = (double*)(hp + P.z1[d]);
        const size_t nn = (size_t)P.n[d] * P.n[d];
        for (size_t i = 0; i < nn; ++i) z[i] = sc * pr.op.A[d][i];
      }
      // node-sum weights w_q theta_q^j / j! (Algorithm 1)
      double* c = (double*)(hp + P.coef);
      for (int j = 0; j < pr.p; ++j) {
        double fact = 1.0;
        for (int k = 2; k <= j; ++k) fact *= k;
        for (int q = 0; q < P.pp.m; ++q) c[(size_t)j * P.pp.m + q] = P.w[q] * std::pow(P.theta[q], j) / fact;
      }
    }
    std::memcpy(hp + S.st_off, S.b.st.data(), S.b.st.size() * sizeof(BatchStage));
    if (!S.b.tj.empty()) std::memcpy(hp + S.tj_off, S.b.tj.data(), S.b.tj.size() * sizeof(BatchTaylor));
    PHIQ_TRY(batch_fetch(h, slot, up, S.up_bytes, stream));

    BatchArgs a{};
    a.st = (const BatchStage*)(up + S.st_off);
    a.tj = (const BatchTaylor*)(up + S.tj_off);
    if (opt.batch_persistent) {
      // one launch; its counters arrive zeroed with the upload
      BatchPersistArgs pa{};
      pa.ctl = (BatchPersistCtl*)(up + S.pc_off);
      pa.done = (unsigned*)(up + S.pc_off + al(sizeof(BatchPersistCtl)));
      pa.total = S.b.total;
      pa.nstages = (int)S.b.st.size();
      pa.spin_limit = kPersistSpinLimit;
      a.stage_begin = 0;
      a.stage_end = pa.nstages;
      a.tile_begin = 0;
      a.tile_end = S.b.total;
      PHIQ_HIP(launch_batch_persistent(a, pa, stream));
      int eslot = 0;
      void* ehost = nullptr;
      PHIQ_TRY(batch_stage(h, sizeof(BatchPersistCtl), &eslot, &ehost));
      PHIQ_HIP(hipMemcpyAsync(ehost, pa.ctl, sizeof(BatchPersistCtl), hipMemcpyDeviceToHost, stream));
      PHIQ_HIP(hipStreamSynchronize(stream));
      if (((const BatchPersistCtl*)ehost)->err) return PHIQ_ERR_HIP;
    } else {
      for (const Launch& L : S.b.launches) {
        a.stage_begin = L.stage_begin;
        a.stage_end = L.stage_end;
        a.tile_begin = L.tile_begin;
        a.tile_end = L.tile_end;
        const long long T = L.tile_end - L.tile_begin;
        const long long blocks = std::min<long long>((T + 7) / 8 * 8, kBatchGrid);
        const BatchStage& s0 = S.b.st[L.stage_begin];
        PHIQ_HIP(launch_batch(a, L.type, s0.np, s0.vec, (int)blocks, stream));
      }
    }
    for (const auto& P : S.pl) {
      phiq_report* rep = P.pr->rep;
      if (!rep) continue;
      std::memset(rep, 0, sizeof(*rep));
      rep->l = P.pp.l;
      rep->m = P.pp.m;
      rep->alpha = P.pp.alpha;
      rep->log10_bound = P.pp.log10_bound;
      rep->selector = P.pp.selector;
      rep->ttm_chains = P.pr->nrhs * ((P.pr->p > 0 ? P.pp.m + P.pp.l * P.pr->p : 0) + 1);
      rep->workspace_bytes = S.total;
      rep->precision_floor = 0.0;  // the one-launch path is FP64
      rep->tol_met = 1;
    }
  }

  // problems outside the persistent path: one plan each, same stream
  for (int i : S.rest) {
    const phiq_problem& pr = probs[i];
    phiq_plan plan = nullptr;
    phiq_report r{};
    PHIQ_TRY(phiq_plan_create(h, &pr.op, pr.t, pr.p, pr.tol, &opt, &plan, &r, stream));
    const phiq_status s = phiq_plan_execute(plan, pr.v, pr.nrhs, pr.out, &r, stream);
    phiq_plan_destroy(plan);
    if (s != PHIQ_OK) return s;
    if (pr.rep) *pr.rep = r;
  }
  if (!S.rest.empty()) PHIQ_HIP(hipStreamSynchronize(stream));
  return PHIQ_OK;
}
