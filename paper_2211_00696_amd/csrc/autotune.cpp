// Tile autotuner and forced tile shapes of the mode products, and the live
// kernel-timing entry points.
#include "engine.h"

extern "C" {

phiq_status phiq_profile_start(phiq_handle h, unsigned class_mask) {
  if (!h) return PHIQ_ERR_INVALID_ARG;
  h->prof.mask = class_mask ? class_mask : ~0u;
  h->prof.recs.clear();
  h->prof.next = 0;
  h->prof.on = true;
  h->prof.open = true;
  return PHIQ_OK;
}

phiq_status phiq_profile_enable(phiq_handle h, int on) {
  if (!h || !h->prof.open) return PHIQ_ERR_INVALID_ARG;
  h->prof.on = on != 0;
  return PHIQ_OK;
}

phiq_status phiq_profile_stop(phiq_handle h, phiq_kernel_stat* stats, int max_stats, int* n_stats) {
  if (!h || (max_stats > 0 && !stats) || max_stats < 0) return PHIQ_ERR_INVALID_ARG;
  DeviceGuard g(h->device);
  h->prof.on = false;
  h->prof.open = false;
  PHIQ_HIP(hipDeviceSynchronize());
  phiq_kernel_stat agg[K_NCLASS];
  std::memset(agg, 0, sizeof(agg));
  for (int c = 0; c < K_NCLASS; ++c) std::strncpy(agg[c].name, kProfClass[c], sizeof(agg[c].name) - 1);
  for (const auto& r : h->prof.recs) {
    float ms = 0.f;
    if (hipEventElapsedTime(&ms, r.e0, r.e1) != hipSuccess) return PHIQ_ERR_HIP;
    agg[r.cls].launches += 1;
    agg[r.cls].ms += ms;
    agg[r.cls].flops += r.flops;
    agg[r.cls].bytes += r.bytes;
  }
  h->prof.recs.clear();
  h->prof.next = 0;
  int k = 0;
  for (int c = 0; c < K_NCLASS; ++c)
    if (agg[c].launches > 0) {
      if (k < max_stats) stats[k] = agg[c];
      ++k;
    }
  if (n_stats) *n_stats = std::min(k, max_stats);
  return PHIQ_OK;
}

phiq_status phiq_tile_config(phiq_handle h, int kind, int cfg, int* count) {
  if (!h || kind < 0 || kind > 7) return PHIQ_ERR_INVALID_ARG;
  const int nc = kind <= 2   ? ttm_num_configs(kind)
                 : kind == 3 ? bf16r_num_configs()
                 : kind == 4 ? bf16r_square_num_configs()
                 : kind == 7 ? f64r_accum_num_configs()
                             : f64r_num_configs();
  if (count) *count = nc;
  if (cfg < -1 || cfg >= nc) return PHIQ_ERR_INVALID_ARG;
  h->force_cfg[kind] = cfg;
  return PHIQ_OK;
}

phiq_status phiq_autotune(phiq_handle h, int dim, const int* n, int p, int m, double* times, hipStream_t st) {
  // times is [64][16] (ms per launch shape and tile shape)
  if (!h || !n || dim < 1 || dim > PHIQ_MAX_DIM || p < 0 || p > PHIQ_MAX_P || m < 1 || m > 4096)
    return PHIQ_ERR_INVALID_ARG;
  long long N = 1;
  for (int d = 0; d < dim; ++d) {
    if (n[d] < 1 || n[d] > PHIQ_MAX_N) return PHIQ_ERR_INVALID_ARG;
    N *= n[d];
  }
  DeviceGuard g(h->device);
  const int nbmax = std::max(m + 1, std::max(p, 1));
  const size_t tb = align_up((size_t)nbmax * N * sizeof(double));
  const size_t eb = align_up((size_t)nbmax * PHIQ_MAX_N * PHIQ_MAX_N / 16 * sizeof(double));
  size_t emax = 0;
  for (int d = 0; d < dim; ++d) emax = std::max(emax, (size_t)nbmax * n[d] * n[d] * sizeof(double));
  const size_t need = 2 * tb + align_up(emax) + align_up((size_t)4 * nbmax * sizeof(double));
  (void)eb;
  PHIQ_TRY(ensure(h, h->ws, need));
  char* wb = (char*)h->ws.p;
  PHIQ_HIP(hipMemsetAsync(wb, 0, need, st));
  double* X = (double*)wb;
  double* O = (double*)(wb + tb);
  double* E = (double*)(wb + 2 * tb);
  double* coef = (double*)(wb + 2 * tb + align_up(emax));
  hipEvent_t e0, e1;
  PHIQ_HIP(hipEventCreate(&e0));
  PHIQ_HIP(hipEventCreate(&e1));
  // the launch shapes of a phi-action: store (nodes + phi_0, and p RHS),
  // node sum, squaring; every axis in turn is the contracted one
  struct Shape {
    int kind, M, L, nb;
  };
  std::vector<Shape> shapes;
  for (int d = 0; d < dim; ++d) {
    const int L = (int)(N / n[d]);
    shapes.push_back({0, n[d], L, m + 1});  // node chains with phi_0's (Gauss)
    shapes.push_back({0, n[d], L, 1});  // phi_0
    if (p > 0 && p != m && p != 1) shapes.push_back({0, n[d], L, p});  // squaring orders
    if (d == 0 && p > 0) {
      shapes.push_back({1, n[d], L, m});
      shapes.push_back({2, n[d], L, p});
    }
  }
  int ti = 0;
  for (const auto& sh : shapes) {
    TtmArgs a{};
    a.E = E;
    a.es = 0;
    a.X = X;
    a.xs = N;
    a.O = O;
    a.os = N;
    a.M = a.K = sh.M;
    a.L = sh.L;
    a.nbatch = sh.nb;
    a.coef = coef;
    a.ldcoef = sh.nb;
    a.np = std::min(4, std::max(1, p));
    a.Y = O;
    a.ys = N;
    a.Yprev = X;
    a.yps = N;
    for (int k = 0; k <= PHIQ_MAX_P; ++k) a.ifact[k] = 1.0;
    int best = -1;
    float best_ms = 1e30f;
    for (int c = 0; c < ttm_num_configs(sh.kind); ++c) {
      if (launch_kind(sh.kind, a, PHIQ_PREC_FP64, st, c) != hipSuccess) continue;  // warm-up
      PHIQ_HIP(hipEventRecord(e0, st));
      const int reps = 3;
      for (int r = 0; r < reps; ++r)
        if (launch_kind(sh.kind, a, PHIQ_PREC_FP64, st, c) != hipSuccess) return PHIQ_ERR_HIP;
      PHIQ_HIP(hipEventRecord(e1, st));
      PHIQ_HIP(hipEventSynchronize(e1));
      float ms = 0.f;
      PHIQ_HIP(hipEventElapsedTime(&ms, e0, e1));
      ms /= reps;
      if (times && ti < 64 && c < 16) times[ti * 16 + c] = ms;
      if (ms < best_ms) {
        best_ms = ms;
        best = c;
      }
    }
    if (best >= 0) {
      const int nbk = sh.kind == 1 ? 1 : sh.nb;
      bool found = false;
      for (auto& e : h->tune)
        if (e.kind == sh.kind && e.M == sh.M && e.L == sh.L && e.nb == nbk) {
          e.cfg = best;
          found = true;
        }
      if (!found) h->tune.push_back({sh.kind, sh.M, sh.L, nbk, best});
    }
    ++ti;
  }
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  return PHIQ_OK;
}

}  // extern "C"
