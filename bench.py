#!/usr/bin/env python3
"""Benchmark: phi_k(-tA)v, k = 0..3, for a 3D advection-diffusion Kronecker sum.

Workload (default): A = A^0 (+) A^1 (+) A^2, A^d = a_d tridiag(-1,2,-1)/h^2 +
b_d tridiag(-1,1,0)/h on n = 256 interior points per axis (N = 16,777,216),
a_d log-uniform in [0.1, 10], b_d uniform in [0, 50] (seed 0), t = 1e-3,
v ~ N(0, 1), Gauss-Legendre nodes, tolerance 1e-8.  The headline is the
plain FP64 method; the same line carries the FP32 and split-bf16 forms of
the mode products on the same problem and (l, m) ("forms": rate, roofline
fraction, relative error per phi_k against the oracle), and the median over
16 coefficient draws of the n = 128 problem ("c2_seeds_median").

One step = one full phi-action through the C ABI (phiq_action): norm bound,
parameter selection, rule, 1D exponentials, quadrature with fused node
sums, modified squaring, phi_0.  Inputs are resident in HBM before the timed
region.  Kernel times come from HIP events the library records on its
launch stream during the timed region.

Prints one JSON line.
"""
from __future__ import annotations

import argparse
import hashlib
import math
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

METRIC = "φ_k(tA)v grid-pts/s + MFMA util: split-BF16 vs FP64 at rel err 1e-8"
PEAK_TFLOPS = {"fp64": 78.6, "fp32": 157.3, "bf16x3": 2500.0, "int8": 5000.0}
HBM_PEAK_GBS = 8000.0


def kernel_source_digest():
    h = hashlib.sha256()
    for f in ("kernels.hip", "tile_fp64.h", "kernels_lowp.hip", "kernels_bf16r.hip", "kernels_f32r.hip", "kernels_f64r.hip", "kernels_i8.hip", "kernels_slab.hip"):
        p = os.path.join(ROOT, "paper_2211_00696_amd", "csrc", f)
        if os.path.exists(p):
            h.update(open(p, "rb").read())
    return h.hexdigest()[:16]


def traffic_key(kernel, precision):
    """Entry name in profiles/traffic.json: the class, suffixed by the precision form unless FP64."""
    return kernel if precision == "fp64" else "%s@%s" % (kernel, precision)


def headline_workload(n, N, seed, rule, precision):
    """config.workload of the advection-diffusion phi-action lines."""
    return ("3D advection-diffusion Kronecker sum, n=%d per axis (N=%d), a_d log-U[0.1,10], "
            "b_d U[0,50], t=1e-3, phi_0..phi_3, v~N(0,1) seed %d, %s, tol 1e-8, %s mode products"
            % (n, N, seed, "Gauss-Legendre" if rule == "gauss" else "adaptive Clenshaw-Curtis", precision.upper()))


def load_traffic(kernel, digest, precision, workload):
    """HBM bytes per launch from committed rocprofv3 counter runs: only from an entry taken on the same
    kernel sources and the same workload (sizes, coefficients, rule, precision form)."""
    p = os.path.join(ROOT, "profiles", "traffic.json")
    if not os.path.exists(p):
        return None
    try:
        d = json.load(open(p))
        ent = d.get(traffic_key(kernel, precision))
        if not ent or ent.get("kernel_digest") != digest or ent.get("workload") != workload:
            return None
        return float(ent["bytes_per_launch"])
    except Exception:
        return None


def blas_threads():
    try:
        from threadpoolctl import threadpool_info

        return max([i.get("num_threads", 1) for i in threadpool_info() if i.get("user_api") == "blas"] or [1])
    except Exception:
        return os.cpu_count() or 1


def cpu_baseline(pr, out_gpu, min_seconds=10.0, max_runs=8):
    """The oracle's own algorithm (numpy, FP64) on the same input, timed: whole
    phi-actions repeated until about min_seconds of CPU work (at most max_runs)."""
    from oracle import phiquad

    threads = blas_threads()
    secs = []
    while len(secs) < max_runs and (not secs or sum(secs) < min_seconds):
        t0 = time.perf_counter()
        ref = phiquad.phiquadmv(pr["mats"], pr["t"], pr["v"], pr["p"], eps=pr["tol"], beta=1.0)
        secs.append(time.perf_counter() - t0)
    N = pr["v"].size
    med = float(np.median(secs))
    errs = [float(np.max(np.abs(out_gpu[k] - ref[k])) / np.max(np.abs(ref[k]))) for k in range(pr["p"] + 1)]
    return {
        "value": N / med,
        "unit": "grid-pts/s",
        "cores": int(threads),
        "kind": "oracle",
        "sample": "%d full phi-actions (all N = %d points, phi_0..phi_%d each) of the same workload by the oracle's "
                  "numpy quadrature + modified squaring (FP64, BLAS threads = %d), %.2f s in total; value from "
                  "the median run" % (len(secs), N, pr["p"], threads, sum(secs)),
        "seconds": float(sum(secs)),
        "run_seconds": secs,
        "affinity_cores": len(os.sched_getaffinity(0)),
        "cpu_model": cpu_model(),
    }, errs


def cpu_model():
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return None


def main():
    ap = argparse.ArgumentParser(description=__doc__, formatter_class=argparse.RawDescriptionHelpFormatter)
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=30)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--n", type=int, default=None,
                    help="grid points per axis (default: 256 for advdiff3d and precision256, 128 for seeds and combo)")
    ap.add_argument("--rule", default="gauss", choices=["gauss", "cc"])
    ap.add_argument("--precision", default="fp64", choices=["fp64", "fp32", "bf16x3", "int8"])
    ap.add_argument("--seed", type=int, default=0)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-autotune", action="store_true")
    ap.add_argument("--slab-products", type=int, default=0, choices=[0, 1, 2],
                    help="phiq_options.slab_products: 0 one axis per pass (default), "
                         "1 two-axis slab products for single-vector chains, 2 for every chain")
    ap.add_argument("--workload", default="advdiff3d",
                    choices=["advdiff3d", "batch512", "combo", "etdrk4", "precision256", "problem1", "problem3",
                             "seeds"],
                    help="advdiff3d: one 3D problem (default); batch512: 512 mixed 2D/3D problems in one "
                         "batched call (phiq_action_batched); etdrk4: 100 ETD-RK4 steps of Allen-Cahn on 3D n=128")
    ap.add_argument("--count", type=int, default=None,
                    help="batch512: number of problems (default 512); seeds: number of coefficient draws (default 16)")
    ap.add_argument("--event-every", type=int, default=10,
                    help="advdiff3d: in the timed region, the dominant kernel class's launches of every this-many-th "
                         "step (the first, the 1+S-th, ...) carry HIP events; 1 = every step")
    ap.add_argument("--batch-persistent", action="store_true",
                    help="batch512: the whole batch in one persistent launch (phiq_options.batch_persistent)")
    ap.add_argument("--no-forms", action="store_true",
                    help="advdiff3d, FP64: skip the FP32 / split-bf16 legs and the n = 128 seed median")
    ap.add_argument("--copy-probe-mib", type=int, default=0,
                    help="before the steps, negate a buffer of this many MiB into another once (a plain device copy "
                         "of known size that calibrates hardware byte counters taken over the same run)")
    args = ap.parse_args()

    if args.n is None:
        args.n = 256 if args.workload in ("advdiff3d", "precision256") else 128
    if args.gpus != 1:
        print(json.dumps({"error": "this benchmark runs on one GPU only; --gpus %d is not supported "
                                   "(the phi-action of one problem is not split across GPUs here)" % args.gpus}))
        sys.exit(2)
    rank = int(os.environ.get("RANK", "0"))

    import torch

    if args.workload == "batch512":
        return bench_batch(args, rank)
    if args.workload == "etdrk4":
        return bench_etd(args, rank)
    if args.workload == "precision256":
        return bench_precision(args, rank)
    if args.workload == "problem1":
        return bench_problem1(args, rank)
    if args.workload == "problem3":
        return bench_problem3(args, rank)
    if args.workload == "seeds":
        return bench_seeds(args, rank)
    if args.workload == "combo":
        return bench_combo(args, rank)

    from paper_2211_00696_amd import inputs, phiq

    assert torch.cuda.is_available(), "bench.py needs a GPU"
    dev = torch.device("cuda:0")
    pr = inputs.problem("advdiff3d", seed=args.seed, n=args.n)
    N = pr["v"].size
    p = pr["p"]
    v = torch.from_numpy(pr["v"]).to(dev)
    out = torch.empty((p + 1, N), dtype=torch.float64, device=dev)
    stream = torch.cuda.current_stream()
    h = phiq.Handle(0)
    opts = dict(rule=args.rule, precision=args.precision, slab_products=args.slab_products,
                accept_floor=args.precision in ("fp32", "bf16x3"))
    if args.copy_probe_mib > 0:
        src = torch.ones(args.copy_probe_mib << 17, dtype=torch.float64, device=dev)
        dst = torch.empty_like(src)
        torch.cuda.synchronize()
        torch.neg(src, out=dst)  # one elementwise kernel: reads and writes copy_probe_mib MiB
        torch.cuda.synchronize()
        del src, dst

    # tile shapes for this problem's launch shapes (autotuner, before timing)
    _, rep0 = h.action(pr["mats"], pr["t"], p, v, tol=pr["tol"], out=out, **opts)
    tuned = None
    if args.precision == "fp64" and not args.no_autotune:
        tt = h.autotune([args.n] * 3, p, rep0["m"] if args.rule == "gauss" else 25)
        tuned = [[int(np.argmin(np.where(r >= 0, r, np.inf))), float(np.min(r[r >= 0]))] for r in tt]
    for _ in range(args.warmup):
        h.action(pr["mats"], pr["t"], p, v, tol=pr["tol"], out=out, **opts)
    torch.cuda.synchronize()

    # which kernel dominates: one step with every launch bracketed
    h.profile_start()
    h.action(pr["mats"], pr["t"], p, v, tol=pr["tol"], out=out, **opts)
    all_stats = h.profile_stop()
    dom = max(all_stats.items(), key=lambda kv: kv[1]["ms"])[0]

    # timed region: K full phi-actions; the dominant kernel's launches in every
    # S-th step are bracketed by HIP events on its launch stream (a bracketed
    # launch leaves the GPU idle for some microseconds, so bracketing every
    # one would slow the steps being timed)
    every = max(1, args.event_every)
    h.profile_start([dom])
    ev0 = torch.cuda.Event(enable_timing=True)
    ev1 = torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    ev0.record(stream)
    rep = None
    for i in range(args.steps):
        if every > 1:
            h.profile_enable(i % every == 0)
        _, rep = h.action(pr["mats"], pr["t"], p, v, tol=pr["tol"], out=out, **opts)
    ev1.record(stream)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    stats = h.profile_stop()
    ms_per_step = wall * 1e3 / args.steps
    ms_events = ev0.elapsed_time(ev1) / args.steps

    # the same steps with no brackets at all, and execute-only with a reused plan
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    for _ in range(args.steps):
        h.action(pr["mats"], pr["t"], p, v, tol=pr["tol"], out=out, **opts)
    torch.cuda.synchronize()
    ms_unprofiled = (time.perf_counter() - t1) * 1e3 / args.steps
    plan = h.plan(pr["mats"], pr["t"], p, tol=pr["tol"], **opts)
    plan.execute(v)
    torch.cuda.synchronize()
    t2 = time.perf_counter()
    for _ in range(args.steps):
        plan.execute(v, out=out.view(1, p + 1, N))
    torch.cuda.synchronize()
    ms_execute = (time.perf_counter() - t2) * 1e3 / args.steps
    plan.close()

    st = stats[dom]
    avg_ms = st["ms"] / st["launches"]
    flops_per_launch = st["flops"] / st["launches"]
    achieved = flops_per_launch / (avg_ms * 1e-3) / 1e12
    fp64_equivalent = achieved
    if args.precision == "int8":
        # executed int8 operations: every kept digit pair, S (S + 1) / 2 of them
        digits = 5 if pr["tol"] >= 1e-6 else (6 if pr["tol"] >= 1e-9 else 7)
        achieved *= digits * (digits + 1) / 2
    peak = PEAK_TFLOPS[args.precision]
    gbs = st["bytes"] / st["launches"] / (avg_ms * 1e-3) / 1e9
    # split bf16: three products at the 2.5 PF bf16 peak leave the kernel far from
    # its matrix roofline; its bound is the FP32 intermediates' HBM traffic
    bound = "hbm" if args.precision == "bf16x3" else "mfma"
    digest = kernel_source_digest()
    workload = headline_workload(args.n, N, args.seed, args.rule, args.precision)
    # the counter runs were taken without the slab products
    traffic = None if args.slab_products else load_traffic(dom, digest, args.precision, workload)
    ttm_total = {k: v for k, v in all_stats.items() if k.startswith("ttm")}
    ttm_ms = sum(s["ms"] for s in ttm_total.values())
    ttm_tflops = sum(s["flops"] for s in ttm_total.values()) / (ttm_ms * 1e-3) / 1e12

    out_host = out.cpu().numpy()
    result = {
        "metric": METRIC,
        "value": N / (ms_per_step * 1e-3),
        "unit": "grid-pts/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms_per_step,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": {"fp64": "f64", "fp32": "f32", "bf16x3": "bf16x3", "int8": "i8"}[args.precision],
        "data": "synthetic",
        "config": {
            "workload": workload,
            "n": args.n, "N": N, "p": p, "t": pr["t"], "tol": pr["tol"], "rule": args.rule,
            "precision": args.precision, "seed": args.seed, "slab_products": args.slab_products,
            "coefficients": pr["coef"],
        },
        "roofline": {
            "kernel": dom,
            "bound": bound,
            "achieved": achieved if bound == "mfma" else gbs,
            "peak": peak if bound == "mfma" else HBM_PEAK_GBS,
            "unit": ("TOP/s" if args.precision == "int8" else "TFLOP/s") if bound == "mfma" else "GB/s",
            "frac": (achieved / peak) if bound == "mfma" else gbs / HBM_PEAK_GBS,
            "mfma_tflops": achieved,
            "mfma_peak_tflops": peak,
            "fp64_equivalent_tflops": fp64_equivalent,
            "traffic": traffic,
            "avg_launch_ms": avg_ms,
            "launches": st["launches"],
            "flops_per_launch": flops_per_launch,
            "algorithmic_bytes_per_launch": st["bytes"] / st["launches"],
        },
        "plan": {"l": rep["l"], "m": rep["m"], "alpha": rep["alpha"], "ttm_chains": rep["ttm_chains"],
                 "log10_bound": rep["log10_bound"]},
        "event_every": every,
        "event_steps": len(range(0, args.steps, every)),
        "ms_per_step_events": ms_events,
        "ms_per_step_unprofiled": ms_unprofiled,
        "ms_per_execute_reused_plan": ms_execute,
        "all_mode_products_tflops": ttm_tflops,
        "kernels_one_step": {k: {"launches": s["launches"], "ms": s["ms"],
                        "tflops": (s["flops"] / (s["ms"] * 1e-3) / 1e12) if s["ms"] > 0 else None,
                        "gbs": (s["bytes"] / (s["ms"] * 1e-3) / 1e9) if s["ms"] > 0 else None}
                    for k, s in all_stats.items()},
        "kernel_digest": digest,
        "autotuned": args.precision == "fp64" and not args.no_autotune,
        "autotune_choice_ms": tuned,
    }
    form_outs = {}
    if args.precision == "fp64" and not args.no_forms:
        result["forms"] = {}
        for prec in ("fp32", "bf16x3"):
            wl = None if args.slab_products else headline_workload(args.n, N, args.seed, args.rule, prec)
            f, o = time_form(h, pr, prec, v, out, max(5, args.steps // 2), args.warmup, ms_per_step, wl,
                             rule=args.rule, slab_products=args.slab_products)
            result["forms"][prec] = f
            form_outs[prec] = o
        result["c2_seeds_median"] = seeds_median(h, args)
    if not args.no_cpu_baseline and rank == 0:
        cb, errs = cpu_baseline(pr, out_host)
        result["cpu_baseline"] = cb
        # every output against the oracle's quadrature at eps = 1e-14
        from oracle import phiquad

        t_ref = time.perf_counter()
        ref = phiquad.phiquadmv(pr["mats"], pr["t"], pr["v"], p, eps=1e-14, beta=1.0)
        t_ref = time.perf_counter() - t_ref
        result["rel_err_vs_oracle_per_phi_k"] = rel_errs(out_host, ref)
        result["oracle_reference"] = {"eps": 1e-14, "seconds": t_ref}
        for prec, o in form_outs.items():
            e = rel_errs(o, ref)
            result["forms"][prec]["rel_err_vs_oracle_per_phi_k"] = e
            result["forms"][prec]["meets_tol"] = bool(max(e) < pr["tol"])
    else:
        result["cpu_baseline"] = None
    h.close()
    if rank == 0:
        print(json.dumps(result), flush=True)


def rel_errs(o, ref):
    return [float(np.max(np.abs(o[k] - ref[k])) / np.max(np.abs(ref[k]))) for k in range(ref.shape[0])]


def time_form(h, pr, prec, v, out, steps, warmup, ms_fp64, workload, **opts):
    """One precision form of the mode products on the headline problem: the same tol (so the same
    (l, m) as FP64; the form's rounding floor is accepted, its error is reported), wall time per
    full phi-action over `steps` unprofiled calls, then one call with every launch timed by HIP
    events for the dominant class's roofline (split bf16: HBM bytes; FP32: the FP32 matrix peak).
    workload names the counter runs the traffic entry must come from (None: no traffic)."""
    import torch

    p = pr["p"]
    N = pr["v"].size
    kw = dict(opts, precision=prec, accept_floor=True)
    for _ in range(warmup):
        h.action(pr["mats"], pr["t"], p, v, tol=pr["tol"], out=out, **kw)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    rep = None
    for _ in range(steps):
        _, rep = h.action(pr["mats"], pr["t"], p, v, tol=pr["tol"], out=out, **kw)
    torch.cuda.synchronize()
    ms = (time.perf_counter() - t0) * 1e3 / steps
    h.profile_start()
    h.action(pr["mats"], pr["t"], p, v, tol=pr["tol"], out=out, **kw)
    stats = h.profile_stop()
    dom = max(stats.items(), key=lambda kv: kv[1]["ms"])[0]
    st = stats[dom]
    avg_ms = st["ms"] / st["launches"]
    tflops = st["flops"] / st["launches"] / (avg_ms * 1e-3) / 1e12
    gbs = st["bytes"] / st["launches"] / (avg_ms * 1e-3) / 1e9
    if prec == "bf16x3":
        # three bf16 products per FP64-equivalent product; bound by the FP32
        # intermediates' HBM traffic
        roof = {"kernel": dom, "bound": "hbm", "achieved": gbs, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                "frac": gbs / HBM_PEAK_GBS, "mfma_tflops_bf16": 3 * tflops,
                "mfma_frac_bf16": 3 * tflops / PEAK_TFLOPS["bf16x3"]}
    else:
        roof = {"kernel": dom, "bound": "mfma", "achieved": tflops, "peak": PEAK_TFLOPS[prec], "unit": "TFLOP/s",
                "frac": tflops / PEAK_TFLOPS[prec], "gbs": gbs}
    roof["traffic"] = load_traffic(dom, kernel_source_digest(), prec, workload) if workload else None
    roof.update({"avg_launch_ms": avg_ms, "launches": st["launches"], "fp64_equivalent_tflops": tflops,
                 "algorithmic_bytes_per_launch": st["bytes"] / st["launches"]})
    torch.cuda.synchronize()
    return {
        "grid_pts_per_s": N / (ms * 1e-3),
        "ms_per_step": ms,
        "steps": steps,
        "speedup_vs_fp64": ms_fp64 / ms,
        "tol": pr["tol"],
        "precision_floor": rep["precision_floor"],
        "tol_met_by_floor": bool(rep["tol_met"]),
        "plan": {"l": rep["l"], "m": rep["m"]},
        "roofline": roof,
        "kernels_one_step": {k: {"launches": s["launches"], "ms": s["ms"]} for k, s in stats.items()},
    }, out.cpu().numpy()


def grouped_ms(call, calls, groups=3):
    """Per-call milliseconds of `call`, run back to back in `groups` groups of calls / groups calls
    (at least one): the median group, so that a one-off stall of the host or of one call shifts one
    group only; the groups' values are returned too."""
    import torch

    per = max(1, calls // groups)
    gms = []
    for _ in range(groups):
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(per):
            call()
        torch.cuda.synchronize()
        gms.append((time.perf_counter() - t0) * 1e3 / per)
    return float(np.median(gms)), gms


def seeds_median(h, args, count=16, n=128, steps=30, warmup=2):
    """The 3D n = 128 problem (FP64, the rule of the headline) over coefficient draws 0..count-1:
    grid points per second of full phi-actions per draw and their median."""
    import torch

    from paper_2211_00696_amd import inputs

    rows = []
    for seed in range(count):
        pr = inputs.problem("advdiff3d", seed=seed, n=n)
        v = torch.from_numpy(pr["v"]).cuda()
        out = torch.empty((pr["p"] + 1, v.numel()), dtype=torch.float64, device="cuda")
        rep = None
        for _ in range(warmup):
            _, rep = h.action(pr["mats"], pr["t"], pr["p"], v, tol=pr["tol"], out=out, rule=args.rule)
        ms, gms = grouped_ms(lambda: h.action(pr["mats"], pr["t"], pr["p"], v, tol=pr["tol"], out=out,
                                              rule=args.rule), steps)
        rows.append({"seed": seed, "alpha": rep["alpha"], "l": rep["l"], "m": rep["m"],
                     "grid_pts_per_s": v.numel() / (ms * 1e-3), "group_ms": gms})
        del v, out
    return {"workload": "3D advection-diffusion n=%d (N=%d), coefficient draws 0..%d, FP64, %s, tol 1e-8, "
                        "the median of three groups of %d back-to-back calls per draw"
                        % (n, n ** 3, count - 1, args.rule, max(1, steps // 3)),
            "median_grid_pts_per_s": float(np.median([r["grid_pts_per_s"] for r in rows])),
            "per_seed": rows}


def ttm_flops(pr, rep):
    """Algorithmic flops of one phi-action: 2 d n N per Kronecker chain, (m + l p + 1) chains, plus the
    1D exponentials (powers, Taylor sums, squarings) counted as 2 n^3 per n x n product."""
    N = pr["v"].size
    n = [m.shape[0] for m in pr["mats"]]
    chain = sum(2.0 * nd * N for nd in n)
    return chain * rep["ttm_chains"]


def bench_batch(args, rank):
    """512 independent problems (dim 2/3, n 16..192, p 1..4, t log-U[1e-4, 1e-1]) per call."""
    import torch

    from paper_2211_00696_amd import inputs, phiq

    probs = inputs.batch_mix(seed=args.seed, count=args.count or 512)
    Ns = [p["v"].size for p in probs]
    Ntot = int(sum(Ns))
    vbuf = torch.empty(Ntot, dtype=torch.float64, device="cuda")
    off = 0
    views = []
    for p, N in zip(probs, Ns):
        vbuf[off:off + N].copy_(torch.from_numpy(p["v"]))
        views.append(vbuf[off:off + N])
        off += N
    outs = [torch.empty((1, p["p"] + 1, N), dtype=torch.float64, device="cuda") for p, N in zip(probs, Ns)]
    bp = [dict(mats=p["mats"], t=p["t"], p=p["p"], tol=p["tol"], v=v, out=o) for p, v, o in zip(probs, views, outs)]
    h = phiq.Handle(0)
    info = phiq.batch_info([dict(mats=p["mats"], t=p["t"], p=p["p"], tol=p["tol"], v_ptr=v.data_ptr(),
                                 out_ptr=o.data_ptr()) for p, v, o in zip(probs, views, outs)])
    bkw = dict(batch_persistent=True) if args.batch_persistent else {}
    _, reps = h.action_batched(bp, **bkw)
    torch.cuda.synchronize()
    for _ in range(args.warmup):
        h.action_batched(bp, **bkw)
    torch.cuda.synchronize()
    stream = torch.cuda.current_stream()
    ev0 = torch.cuda.Event(enable_timing=True)
    ev1 = torch.cuda.Event(enable_timing=True)
    t0 = time.perf_counter()
    ev0.record(stream)
    for _ in range(args.steps):
        h.action_batched(bp, **bkw)
    ev1.record(stream)
    torch.cuda.synchronize()
    wall = (time.perf_counter() - t0) / args.steps
    gpu_ms = ev0.elapsed_time(ev1) / args.steps
    # the same problems one phiq_action call each (for comparison)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    for p, v in zip(probs, views):
        h.action(p["mats"], p["t"], p["p"], v, tol=p["tol"])
    torch.cuda.synchronize()
    seq = time.perf_counter() - t1
    # parity sample: batched vs separate call on a few problems
    errs = []
    for i in range(0, len(probs), max(1, len(probs) // 8)):
        ref, _ = h.action(probs[i]["mats"], probs[i]["t"], probs[i]["p"], views[i], tol=probs[i]["tol"])
        o = outs[i][0]
        errs.append(float(((o - ref).abs().max() / ref.abs().max()).item()))
    flops = sum(ttm_flops(p, r) for p, r in zip(probs, reps))
    peak = PEAK_TFLOPS["fp64"]
    achieved = flops / (gpu_ms * 1e-3) / 1e12
    result = {
        "metric": "phi_k(tA)v grid-pts/s, batch of %d mixed problems in one call" % len(probs),
        "value": Ntot / wall,
        "unit": "grid-pts/s",
        "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
        "ms_per_step": wall * 1e3,
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "f64", "data": "synthetic",
        "config": {"workload": "%d problems: dim 2 or 3 (p=1/2), n uniform in 16..192, p uniform in 1..4, "
                               "t log-uniform in [1e-4, 1e-1], a_d log-U[0.1,10], b_d U[0,50], v~N(0,1), "
                               "Gauss, tol 1e-8, seed %d" % (len(probs), args.seed),
                   "problems": len(probs), "grid_points": Ntot, "seed": args.seed,
                   "persistent_launch": bool(args.batch_persistent)},
        "roofline": {"kernel": "batch_kernel", "bound": "mfma", "achieved": achieved, "peak": peak,
                     "unit": "TFLOP/s", "frac": achieved / peak, "traffic": None,
                     "flops_per_step": flops, "gpu_ms_per_step": gpu_ms,
                     "note": "mode-product flops only (the 1D exponentials are not counted)"},
        "schedule": info,
        "ms_separate_calls": seq * 1e3,
        "speedup_vs_separate_calls": seq / wall,
        "rel_err_batched_vs_separate_sample": max(errs),
    }
    if not args.no_cpu_baseline and rank == 0:
        from oracle import phiquad

        sample = list(range(0, len(probs), 32))  # every 32nd problem of the batch
        t2 = time.perf_counter()
        pts = 0
        for i in sample:
            pr = probs[i]
            phiquad.phiquadmv(pr["mats"], pr["t"], pr["v"], pr["p"], eps=pr["tol"], beta=1.0)
            pts += Ns[i]
        dt = time.perf_counter() - t2
        result["cpu_baseline"] = {"value": pts / dt, "unit": "grid-pts/s", "cores": blas_threads(),
                                  "kind": "oracle", "sample": "every 32nd problem of the batch (%d problems, "
                                  "%d points) by the oracle's numpy quadrature, %.2f s" % (len(sample), pts, dt)}
    else:
        result["cpu_baseline"] = None
    h.close()
    if rank == 0:
        print(json.dumps(result), flush=True)


def bench_precision(args, rank):
    """3D n=256 advection-diffusion, phi_0..phi_3: every precision form and selector at tol 1e-5, 1e-6
    and 1e-10, error per phi_k against the oracle (its numpy quadrature at eps 1e-14), time per action."""
    import torch

    from oracle import phiquad
    from paper_2211_00696_amd import inputs, phiq, selector

    n = args.n
    pr = inputs.problem("advdiff3d", seed=args.seed, n=n)
    N, p = pr["v"].size, pr["p"]
    v = torch.from_numpy(pr["v"]).cuda()
    h = phiq.Handle(0)
    h.selector_set(selector.load_weights())
    _, rep0 = h.action(pr["mats"], pr["t"], p, v, tol=1e-8)
    h.autotune([n] * 3, p, rep0["m"])
    t0 = time.perf_counter()
    ref = phiquad.phiquadmv(pr["mats"], pr["t"], pr["v"], p, eps=1e-14, beta=1.0)
    oracle_s = time.perf_counter() - t0
    runs = []
    for tol in (1e-5, 1e-6, 1e-10):
        for prec in ("fp64", "fp32", "bf16x3"):
            for sel in ("paper", "mlp"):
                kw = dict(tol=tol, precision=prec, selector=sel, accept_floor=prec != "fp64")
                out, rep = h.action(pr["mats"], pr["t"], p, v, **kw)
                h.action(pr["mats"], pr["t"], p, v, **kw)
                torch.cuda.synchronize()
                t1 = time.perf_counter()
                for _ in range(args.steps):
                    h.action(pr["mats"], pr["t"], p, v, out=out, **kw)
                torch.cuda.synchronize()
                ms = (time.perf_counter() - t1) * 1e3 / args.steps
                o = out.cpu().numpy()
                errs = [float(np.max(np.abs(o[k] - ref[k])) / np.max(np.abs(ref[k]))) for k in range(p + 1)]
                runs.append(dict(tol=tol, precision=prec, selector=sel, ms=ms, grid_pts_per_s=N / (ms * 1e-3),
                                 l=rep["l"], m=rep["m"], selector_used=rep["selector"], rel_err_per_phi_k=errs,
                                 meets_tol=max(errs) <= tol))
                print(json.dumps(runs[-1]), file=sys.stderr, flush=True)
    # FP64 mode-product utilisation at n=256 (live events, one action)
    h.profile_start(["ttm_store", "ttm_accum", "ttm_square"])
    h.action(pr["mats"], pr["t"], p, v, tol=1e-8)
    st = h.profile_stop()
    util = {k: s["flops"] / (s["ms"] * 1e-3) / 1e12 / PEAK_TFLOPS["fp64"] for k, s in st.items() if s["ms"] > 0}
    base = {r["tol"]: r["ms"] for r in runs if r["precision"] == "fp64" and r["selector"] == "paper"}
    speed = []
    for r in runs:
        if r["meets_tol"]:
            speed.append(dict(tol=r["tol"], form=r["precision"] + "+" + r["selector"], speedup_vs_fp64_paper=base[r["tol"]] / r["ms"]))
    best = {}
    for s_ in speed:
        if s_["tol"] not in best or s_["speedup_vs_fp64_paper"] > best[s_["tol"]]["speedup_vs_fp64_paper"]:
            best[s_["tol"]] = s_
    result = {"metric": "phi_k(tA)v grid-pts/s by precision form and selector, 3D n=%d" % n, "unit": "grid-pts/s",
              "n_gpus": 1, "steps": args.steps, "data": "synthetic", "dtype": "f64/f32/bf16x3",
              "config": {"workload": "3D advection-diffusion n=%d (N=%d), t=1e-3, phi_0..phi_3, seed %d" % (n, N, args.seed)},
              "oracle_seconds": oracle_s, "runs": runs, "fp64_mfma_utilisation_tol1e-8": util,
              "meets_tol_speedups": speed, "best_at_equal_accuracy": best}
    h.close()
    if rank == 0:
        print(json.dumps(result), flush=True)


def bench_problem1(args, rank):
    """The paper's Problem 1 (Section 4): 3D heat, n = 2^r - 1, tau = 1/8, b = sin sin sin, phi_1..phi_20,
    eps 1e-14, Gauss and Clenshaw-Curtis: our time per action next to the paper's (one thread of an
    Intel i5-8279U, MATLAB), with the error against the closed form."""
    import torch

    from paper_2211_00696_amd import inputs, phiq

    paper = {4: (0.19, 0.11), 5: (0.95, 1.15), 6: (1.34, 1.79), 7: (25.63, 31.50)}
    h = phiq.Handle(0)
    rows = []
    for r in (4, 5, 6, 7):
        n = 2 ** r - 1
        pr = inputs.problem("heat3d_eig", n=n)
        v = torch.from_numpy(pr["v"]).cuda()
        lam = 3.0 * 4.0 * (n + 1) ** 2 * math.sin(math.pi / (2 * (n + 1))) ** 2
        for rule in ("gauss", "cc"):
            out, rep = h.action(pr["mats"], pr["t"], pr["p"], v, tol=pr["tol"], rule=rule)
            h.action(pr["mats"], pr["t"], pr["p"], v, tol=pr["tol"], rule=rule)
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            for _ in range(args.steps):
                h.action(pr["mats"], pr["t"], pr["p"], v, tol=pr["tol"], rule=rule, out=out)
            torch.cuda.synchronize()
            ms = (time.perf_counter() - t0) * 1e3 / args.steps
            # phi_k(-tau A) b = phi_k(-tau lam) b exactly (b is an eigenvector)
            from oracle import phi_exact

            o = out.cpu().numpy()
            err = max(float(np.max(np.abs(o[k] - phi_exact.phi_scalar(k, -pr["t"] * lam) * pr["v"]))
                            / np.max(np.abs(phi_exact.phi_scalar(k, -pr["t"] * lam) * pr["v"]))) for k in range(1, pr["p"] + 1))
            rows.append(dict(r=r, N=n ** 3, rule=rule, l=rep["l"], m=rep["m"] if rule == "gauss" else None,
                             ms=ms, paper_seconds=paper[r][0 if rule == "gauss" else 1],
                             ratio_paper_over_ours=paper[r][0 if rule == "gauss" else 1] / (ms * 1e-3),
                             max_rel_err_phi_1_to_20=err))
    h.close()
    if rank == 0:
        print(json.dumps({"metric": "Problem 1 (Section 4) time per phi_1..phi_20 action vs the paper",
                          "unit": "ms", "note": "paper: serial MATLAB on one thread of an Intel i5-8279U "
                          "(context, another machine)", "rows": rows}), flush=True)


# Tables TimesHochOster7 / TimesHochOster8 (seconds; Gauss, CC) per method and step count
PAPER_P3 = {
    127: {1: {2: (0.14, 0.17), 8: (0.12, 0.21), 32: (0.42, 0.77), 128: (1.23, 2.88), 512: (4.55, 11.15)},
          2: {2: (0.10, 0.15), 8: (0.22, 0.40), 32: (0.67, 1.55), 128: (2.42, 5.69), 512: (8.94, 22.22)},
          3: {2: (0.18, 0.41), 8: (0.57, 1.37), 32: (1.95, 5.19), 128: (6.56, 20.29), 512: (25.17, 78.17)}},
    255: {1: {2: (0.13, 0.25), 8: (0.38, 0.78), 32: (1.32, 2.87), 128: (4.87, 11.07), 512: (19.20, 45.55)},
          2: {2: (0.22, 0.41), 8: (0.81, 1.50), 32: (2.56, 5.76), 128: (10.07, 22.51), 512: (38.25, 91.02)},
          3: {2: (0.59, 1.37), 8: (2.10, 5.20), 32: (7.74, 20.65), 128: (28.89, 80.64), 512: (108.33, 305.07)}},
}


def bench_problem3(args, rank):
    """The paper's Problem 3 (Section 5): exponential Euler / RK2 / RK3 on 2D Hochbruck-Ostermann with
    2^7 and 2^8 elements per axis, T = 1: total time per run next to the paper's Tables TimesHochOster7/8,
    and the error against the exact solution."""
    import torch

    from oracle import exprk as OR
    from paper_2211_00696_amd import inputs, phiq

    h = phiq.Handle(0)
    rows = []
    for n in (127, 255):
        mats = [inputs.fd_laplacian(n), inputs.fd_laplacian(n)]
        u0 = torch.from_numpy(OR.exact(n, 0.0)).cuda()
        ue = OR.exact(n, 1.0)
        for method in (1, 2, 3):
            for rule, form in (("gauss", "separate"), ("gauss", "combo"), ("cc", "separate")):
                u = u0.clone()
                h.exprk(mats, method, 2, u, rule=rule, tol=1e-14, form=form)  # warm-up
                for steps in (2, 8, 32, 128, 512):
                    u = u0.clone()
                    torch.cuda.synchronize()
                    t0 = time.perf_counter()
                    h.exprk(mats, method, steps, u, rule=rule, tol=1e-14, form=form)
                    torch.cuda.synchronize()
                    dt = time.perf_counter() - t0
                    err = float(np.max(np.abs(u.cpu().numpy() - ue)))
                    ps = PAPER_P3[n][method][steps][0 if rule == "gauss" else 1]
                    rows.append(dict(elements=n + 1, method=["", "Euler", "RK2", "RK3"][method], rule=rule,
                                     form=form, steps=steps, seconds=dt, paper_seconds=ps, ratio_paper_over_ours=ps / dt,
                                     err_vs_exact=err))
                    print(json.dumps(rows[-1]), file=sys.stderr, flush=True)
    h.close()
    if rank == 0:
        print(json.dumps({"metric": "Problem 3 (Section 5) total time of an exponential Runge-Kutta run, T = 1",
                          "unit": "s", "note": "paper: serial MATLAB on one thread of an Intel i5-8279U "
                          "(context, another machine); tol 1e-14 as in the paper", "rows": rows}), flush=True)


def bench_combo(args, rank):
    """Linear combinations sum_j phi_j(-tA) b_j, j = 0..3, on the 3D n=128 advection-diffusion operator
    (four seeded N(0,1) vectors): one phiq_plan_execute_combo against the four phi_j b_j from separate
    executions of the same plan (summed on the device), per rule and precision; plans reused, times per
    combination after warm-up."""
    import torch

    from paper_2211_00696_amd import inputs, phiq

    pr = inputs.problem("advdiff3d", seed=args.seed, n=args.n)
    N = pr["v"].size
    p = pr["p"]
    g = torch.Generator(device="cuda")
    g.manual_seed(args.seed)
    bs = [torch.randn(N, dtype=torch.float64, device="cuda", generator=g) for _ in range(p + 1)]
    h = phiq.Handle(0)
    rows = []
    steps = max(3, args.steps // 3)
    for rule in ("gauss", "cc"):
        for precision in ("fp64", "fp32", "bf16x3"):
            plan = h.plan(pr["mats"], pr["t"], p, tol=pr["tol"], rule=rule, precision=precision,
                          accept_floor=precision not in ("fp64", "int8"))
            out = torch.empty((1, p + 1, N), dtype=torch.float64, device="cuda")

            def separate():
                acc = torch.zeros(N, dtype=torch.float64, device="cuda")
                for j, b in enumerate(bs):
                    plan.execute(b, out=out)
                    acc += out[0, j]
                return acc

            def timed(fn):
                fn()
                torch.cuda.synchronize()
                t0 = time.perf_counter()
                for _ in range(steps):
                    r = fn()
                torch.cuda.synchronize()
                return (time.perf_counter() - t0) * 1e3 / steps, r

            ms_c, rc = timed(lambda: plan.execute_combo(bs))
            ms_s, rs = timed(separate)
            rep = plan.report
            rows.append(dict(rule=rule, precision=precision, l=rep["l"], m=rep["m"], ms_combo=ms_c,
                             ms_separate=ms_s, speedup=ms_s / ms_c,
                             rel_diff=float((rc - rs).abs().max() / rs.abs().max())))
            print(json.dumps(rows[-1]), file=sys.stderr, flush=True)
            plan.close()
    h.close()
    if rank == 0:
        print(json.dumps({"metric": "linear combination sum_j phi_j(-tA) b_j (j = 0..3), 3D n=128 advection-diffusion",
                          "unit": "ms per combination", "higher_is_better": False,
                          "config": {"workload": "3D advection-diffusion n=%d (N=%d), t=1e-3, tol 1e-8, seed %d, "
                                     "b_j ~ N(0,1)" % (args.n, N, args.seed)},
                          "rows": rows}), flush=True)


def bench_seeds(args, rank):
    """The 3D n=128 benchmark over the coefficient draws of seeds 0..count-1 (--count, default 16):
    per seed the plan and the time of a full phiq_action (Gauss and Clenshaw-Curtis), and the medians."""
    import torch

    from paper_2211_00696_amd import inputs, phiq

    count = args.count or 16
    h = phiq.Handle(0)
    rows = []
    for seed in range(count):
        pr = inputs.problem("advdiff3d", seed=seed, n=args.n)
        N = pr["v"].size
        v = torch.from_numpy(pr["v"]).cuda()
        out = torch.empty((pr["p"] + 1, N), dtype=torch.float64, device="cuda")
        row = dict(seed=seed, coefficients=pr["coef"])
        for rule in ("gauss", "cc"):
            for _ in range(2):
                _, rep = h.action(pr["mats"], pr["t"], pr["p"], v, tol=pr["tol"], out=out, rule=rule)
            ms, gms = grouped_ms(lambda: h.action(pr["mats"], pr["t"], pr["p"], v, tol=pr["tol"], out=out, rule=rule),
                                 args.steps)
            row[rule] = dict(ms=ms, grid_pts_per_s=N / (ms * 1e-3), l=rep["l"], m=rep["m"], alpha=rep["alpha"],
                             group_ms=gms)
        rows.append(row)
        print(json.dumps(row), file=sys.stderr, flush=True)
    h.close()
    med = {r: float(np.median([row[r]["grid_pts_per_s"] for row in rows])) for r in ("gauss", "cc")}
    if rank == 0:
        print(json.dumps({"metric": "phi_k(tA)v grid-pts/s over coefficient draws, 3D n=%d" % args.n,
                          "unit": "grid-pts/s", "seeds": count, "steps": args.steps, "median": med,
                          "rows": rows}), flush=True)


def bench_etd(args, rank):
    """u_t = Lap u + u - u^3 on (0,1)^3, Dirichlet, n = 128 interior points per axis, tau = 0.01,
    u0 ~ U(-1, 1) (seed), 100 ETD-RK4 steps: graph-replayed against directly launched."""
    import torch

    from paper_2211_00696_amd import inputs, phiq

    n, steps, tau = args.n, 100, 0.01
    mats = [inputs.fd_laplacian(n) for _ in range(3)]
    N = n ** 3
    rng = np.random.default_rng(args.seed)
    u0 = torch.from_numpy(rng.uniform(-1.0, 1.0, N)).cuda()
    h = phiq.Handle(0)
    for form in ("combo", "separate"):
        warm = u0.clone()
        h.etdrk4(mats, tau, 2, warm, graph=True, form=form)
    runs = {}
    for mode in ("graph", "direct", "separate"):
        u = u0.clone()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        rep = h.etdrk4(mats, tau, steps, u, graph=(mode != "direct"),
                       form="separate" if mode == "separate" else "combo")
        torch.cuda.synchronize()
        runs[mode] = (time.perf_counter() - t0, rep, u)
    same = bool(torch.equal(runs["graph"][2], runs["direct"][2]))
    us = runs["separate"][2]
    forms_rel = float((runs["graph"][2] - us).abs().max() / us.abs().max())
    wall, rep, u = runs["graph"]
    chains = rep["ttm_chains_per_step"] * steps
    flops = chains * 2.0 * 3 * n * N
    result = {
        "metric": "ETD-RK4 steps/s, Allen-Cahn 3D n=%d" % n,
        "value": steps / wall, "unit": "steps/s", "n_gpus": 1, "steps": steps, "warmup": 2,
        "ms_per_step": wall * 1e3 / steps, "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": "f64", "data": "synthetic",
        "config": {"workload": "u_t = Lap u + u - u^3 on (0,1)^3, Dirichlet FD, n=%d per axis, tau=%g, %d steps, "
                               "u0 ~ U(-1,1) seed %d, tol 1e-8, Gauss, FP64; every stage one linear combination "
                               "sum_j phi_j b_j; the step is captured in a hipGraph and replayed"
                               % (n, tau, steps, args.seed), "n": n, "tau": tau},
        "report": rep,
        "ms_per_step_direct": runs["direct"][0] * 1e3 / steps,
        "graph_equals_direct": same,
        "separate_form": {"ms_per_step": runs["separate"][0] * 1e3 / steps,
                          "ttm_chains_per_step": runs["separate"][1]["ttm_chains_per_step"],
                          "rel_diff_vs_combo": forms_rel},
        "mode_product_tflops": flops / wall / 1e12,
        "max_abs_u": float(u.abs().max()),
        "cpu_baseline": None,
    }
    h.close()
    if rank == 0:
        print(json.dumps(result), flush=True)


if __name__ == "__main__":
    main()
