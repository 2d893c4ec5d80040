// Mode-product launches with their live timing, the autotuned or default
// tile shape per launch shape, the grow-only workspace and the pinned staging
// of uploads.
#include "engine.h"

namespace phiq {

hipEvent_t prof_event(phiq_handle h) {
  Profiler& pr = h->prof;
  if (pr.next < pr.pool.size()) return pr.pool[pr.next++];
  hipEvent_t e = nullptr;
  if (hipEventCreate(&e) != hipSuccess) return nullptr;
  pr.pool.push_back(e);
  pr.next = pr.pool.size();
  return e;
}

// Launch through f() (exactly one kernel); when this class is profiled the
// kernel's dispatch carries a start and a stop event.

void ttm_work(const TtmArgs& a, int cls, double* flops, double* bytes) {
  const double N = (double)a.L * a.K;
  const double no = a.nouter > 1 ? a.nouter : 1;  // independent problems of one launch
  *flops = 2.0 * a.M * a.K * (double)a.L * a.nbatch * no;
  // distinct inputs: one when shared, nbatch / xdiv when grouped
  const double nx = a.xs == 0 ? 1.0 : (a.xdiv > 0 ? (double)((a.nbatch + a.xdiv - 1) / a.xdiv) : (double)a.nbatch);
  const double xin = nx * N * no;
  double out = (double)a.nbatch * a.M * a.L * no;
  double extra = 0.0;
  if (cls == K_TTM_ACCUM) out = (double)a.np * a.M * a.L * no;
  if (cls == K_TTM_SQUARE) extra = (double)(a.nbatch + a.order0) * a.M * a.L * no;  // the y_j read once
  if (a.yacc) extra += out;  // the previous output read back
  const double xb = a.x_f32 ? 4.0 : 8.0;
  const double ob = (a.o_f32 && cls == K_TTM_STORE) ? 4.0 : 8.0;
  const double nf = a.es == 0 ? 0.0 : (a.emod > 0 ? (double)std::min(a.emod, a.nbatch) : (double)a.nbatch);
  *bytes = xb * xin + ob * out + 8.0 * (extra + nf * a.M * a.K);
}

int tuned_cfg(phiq_handle h, int kind, const TtmArgs& a) {
  const int nb = (kind == 1) ? 1 : a.nbatch;
  for (const auto& e : h->tune)
    if (e.kind == kind && e.M == a.M && e.L == a.L && e.nb == nb) return e.cfg;
  return -1;
}

// Without a tuned entry: the shapes the autotuner picks at n = 128 (stores:
// 64 x 128 eight-wave tiles when they fill the GPU, 64 x 64 tiles with
// 32-deep chunks when they would not; node sums: 64 x 64, eight waves;
// squaring: all orders per block, eight waves), else the kernels' defaults.
int fallback_cfg(int kind, const TtmArgs& a) {
  if (kind == 0 && a.M >= 128) {
    const long long tiles = (long long)((a.M + 63) / 64) * ((a.L + 127) / 128) * a.nbatch;
    return tiles < 768 ? 6 : 11;
  }
  if (kind == 1 && a.M >= 128) return 6;  // node sum: 64 x 64 tiles, eight waves
  if (kind == 2 && a.M >= 128 && a.nbatch <= 4 && a.es == 0) return 11;
  return -1;
}

int launch_kind(int kind, const TtmArgs& a, phiq_precision prec, hipStream_t st, int cfg) {
  if (kind == 1) return launch_ttm_accum(a, prec, st, cfg);
  if (kind == 2) return launch_ttm_square(a, prec, st, cfg);
  return launch_ttm_store(a, prec, st, cfg);
}


phiq_status L_ttm(phiq_handle h, int cls, const TtmArgs& a0, phiq_precision prec, hipStream_t st,
                  const TwinMap* tw) {
  double fl, by;
  TtmArgs a = a0;
  a.stop = h->guard;
  if (prec != PHIQ_PREC_FP64) {
    if (!tw) return PHIQ_ERR_INVALID_ARG;
    tw->lookup(a.E, prec, &a.Ea, &a.Eb);
    if (!a.Ea) return PHIQ_ERR_INVALID_ARG;
  }
  double f = 1.0;
  for (int k = 0; k <= PHIQ_MAX_P; ++k) {
    a.ifact[k] = 1.0 / f;
    f *= (k + 1);
  }
  ttm_work(a, cls, &fl, &by);
  const int kind = kind_of(cls);
  // split bf16 and FP32: kinds 3 / 4 force the resident-factor shapes of the
  // plain and the squaring products (0 = the general tile kernel)
  int cfg = (prec != PHIQ_PREC_FP64 && kind != 1) ? h->force_cfg[kind == 0 ? 3 : 4]
            : (prec != PHIQ_PREC_FP64) ? -1
                                       : (h->force_cfg[kind] >= 0 ? h->force_cfg[kind] : tuned_cfg(h, kind, a));
  if (prec == PHIQ_PREC_FP64 && cfg < 0) cfg = fallback_cfg(kind, a);
  // FP64 products: the resident-factor kernels first (kinds 5 / 6 / 7 of
  // phiq_tile_config for plain / squaring / node-sum products), unless a
  // tile shape is forced
  const bool try_r = prec == PHIQ_PREC_FP64 && h->force_cfg[kind] < 0;
  const int rcfg = h->force_cfg[kind == 0 ? 5 : (kind == 2 ? 6 : 7)];
  return prof_launch(h, st, cls, fl, by, [&] {
    if (try_r) {
      const int r = kind == 0   ? launch_ttm_store_f64r(a, st, rcfg)
                    : kind == 2 ? launch_ttm_square_f64r(a, st, rcfg)
                                : launch_ttm_accum_f64r(a, st, rcfg);
      if (r != hipErrorNotSupported) return r;
    }
    return launch_kind(kind, a, prec, st, cfg);
  });
}

phiq_status L_gemm(phiq_handle h, const GemmJob* jobs, int njobs, int nm, hipStream_t st) {
  const double n = nm;
  return prof_launch(h, st, K_GEMM, 2.0 * n * n * n * njobs, 24.0 * n * n * njobs,
                     [&] { return launch_gemm_jobs(jobs, njobs, nm, st, h->guard); });
}

phiq_status L_taylor(phiq_handle h, const TaylorJob* jobs, int njobs, int nm, int K, hipStream_t st) {
  const double n = nm;
  return prof_launch(h, st, K_TAYLOR, 2.0 * K * n * n * njobs, 8.0 * (K + 1) * n * n * njobs,
                     [&] { return launch_taylor_jobs(jobs, njobs, nm, st, h->guard); });
}

phiq_status L_scale(phiq_handle h, const ScaleJob* jobs, int njobs, int nm, hipStream_t st) {
  const double n = nm;
  return prof_launch(h, st, K_SCALE, n * n * njobs, 16.0 * n * n * njobs,
                     [&] { return launch_scale_jobs(jobs, njobs, nm, st, h->guard); });
}

phiq_status ensure(phiq_handle h, DevBuf& b, size_t bytes) {
  if (bytes <= b.cap) return PHIQ_OK;
  const size_t want = align_up(bytes + bytes / 8);
  if (h->cap_bytes && h->held() - b.cap + want > h->cap_bytes) {
    if (h->held() - b.cap + bytes > h->cap_bytes) return PHIQ_ERR_OOM;
  }
  size_t get = want;
  if (h->cap_bytes && h->held() - b.cap + get > h->cap_bytes) get = align_up(bytes);
  if (b.p) {
    PHIQ_HIP(hipDeviceSynchronize());
    PHIQ_HIP(hipFree(b.p));
    b.p = nullptr;
    b.cap = 0;
  }
  if (hipMalloc(&b.p, get) != hipSuccess) {
    b.p = nullptr;
    (void)hipGetLastError();
    return PHIQ_ERR_OOM;
  }
  b.cap = get;
  return PHIQ_OK;
}

// Pinned staging buffer for one host->device copy; waits if the slot's
// previous copy has not run yet.
phiq_status stage_acquire(phiq_handle h, size_t bytes, int* slot, void** host) {
  Staging& s = h->stage;
  const int k = s.next;
  s.next = (s.next + 1) % 3;
  if (s.pending[k]) {
    PHIQ_HIP(hipEventSynchronize(s.ev[k]));
    s.pending[k] = false;
  }
  if (s.cap[k] < bytes) {
    if (s.host[k]) PHIQ_HIP(hipHostFree(s.host[k]));
    s.host[k] = nullptr;
    s.cap[k] = 0;
    const size_t want = align_up(std::max(bytes, (size_t)1 << 16));
    if (hipHostMalloc(&s.host[k], want, hipHostMallocDefault) != hipSuccess) {
      s.host[k] = nullptr;
      return PHIQ_ERR_OOM;
    }
    s.cap[k] = want;
  }
  if (!s.ev[k]) PHIQ_HIP(hipEventCreateWithFlags(&s.ev[k], hipEventDisableTiming));
  *slot = k;
  *host = s.host[k];
  return PHIQ_OK;
}

phiq_status stage_copy(phiq_handle h, int slot, void* dst, size_t bytes, hipStream_t st) {
  PHIQ_HIP(hipMemcpyAsync(dst, h->stage.host[slot], bytes, hipMemcpyHostToDevice, st));
  PHIQ_HIP(hipEventRecord(h->stage.ev[slot], st));
  h->stage.pending[slot] = true;
  return PHIQ_OK;
}

// Staged upload through a kernel that reads the pinned host buffer.
phiq_status stage_fetch(phiq_handle h, int slot, void* dst, size_t bytes, hipStream_t st) {
  PHIQ_HIP(launch_fetch(dst, h->stage.host[slot], bytes, st));
  PHIQ_HIP(hipEventRecord(h->stage.ev[slot], st));
  h->stage.pending[slot] = true;
  return PHIQ_OK;
}

}  // namespace phiq
