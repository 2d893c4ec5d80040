"""Summaries of rocprofv3 CSV output for bench.py runs.

  python -m paper_2211_00696_amd.rocprof_summary times   TRACE.csv BENCH.json
  python -m paper_2211_00696_amd.rocprof_summary traffic FETCH.csv WRITE.csv BENCH.json COPY_MIB
  python -m paper_2211_00696_amd.rocprof_summary mfma   COUNTERS.csv BENCH.json
  python -m paper_2211_00696_amd.rocprof_summary timeline TRACE.csv INDEX
  python -m paper_2211_00696_amd.rocprof_summary batch  TRACE.csv

`batch` takes the last run of consecutive batched-stage kernels
(`batch_kernel`, `batch_wide_kernel`: one phiq_action_batched call) and sums
their time per stage kind, order count and staging width.

`timeline` prints the kernels between the INDEX-th and the next plan upload
(`fetch_kernel`, one per phiq_action call) in start order, with their queue
(stream), and the busy and idle time of the GPU over that window.

`times` reads a `--kernel-trace` CSV and prints a markdown table per kernel,
plus the average duration of the dominant class's launches inside bench.py's
timed region (to compare with the live HIP-event figure in BENCH.json).

`traffic` reads two `--pmc FETCH_SIZE` / `--pmc WRITE_SIZE` counter CSVs of
the same command, calibrates each counter with the plain device copy that
`bench.py --copy-probe-mib COPY_MIB` launches (a negation of COPY_MIB MiB into
another buffer: COPY_MIB MiB read, COPY_MIB MiB written), and prints the HBM
bytes per launch of the dominant class as JSON for profiles/traffic.json
(keyed by the class, suffixed `@fp32` / `@bf16x3` for the reduced forms).

`mfma` reads a `--pmc` counter CSV and prints, for the dominant class's
timed-region launches, every counter's mean per launch; with
SQ_INSTS_VALU_MFMA_MOPS_F64 (or _F32, _BF16) the MFMA flops the hardware
executed (MOPS x 512) next to the algorithmic flops, with MfmaUtil rocprofv3's derived MFMA
utilisation, and with the LDS / wait counters the bank-conflict cycles per
LDS instruction and the wait fractions of the wave cycles.

bench.py's step sequence after warm-up is: K timed actions, K untimed
actions, one plan execution, K executions of the reused plan.  Every step
launches the same kernels, so the timed region's launches of a class are the
K*L launches that precede the last (2K+1)*L, with L the class's launches per
step.
"""
from __future__ import annotations

import csv
import json
import re
import sys
from collections import defaultdict

CLASS_RE = {
    # int8 digit products: modes 0 (digits out) and 1 (FP64 out) count as stores, 2 as squaring
    "ttm_store": re.compile(r"(^|::)ttm_(lp_|bf16r_|f32r_|f64r_)?store_kernel|(^|::)i8_product_kernel<\d+, \d+, [01]>"),
    "ttm_slab": re.compile(r"(^|::)slab2_kernel"),
    "ttm_accum": re.compile(r"(^|::)ttm_(lp_|f64r_)?accum_kernel"),
    "ttm_square": re.compile(r"(^|::)ttm_(lp_|bf16r_|f32r_|f64r_)?square(_all)?_kernel|(^|::)i8_product_kernel<\d+, \d+, 2>"),
    "slice": re.compile(r"(^|::)i8_(slice_rows|absmax|slice_tensor)_kernel"),
    "gemm": re.compile(r"(^|::)gemm_(jobs|panel)_kernel"),
    "taylor": re.compile(r"(^|::)taylor_jobs_kernel"),
    "scale": re.compile(r"(^|::)scale_jobs_kernel"),
    "node_sum": re.compile(r"(^|::)node_sum_kernel"),
    "absdiff": re.compile(r"(^|::)absdiff_max_kernel"),
}
COPY_RE = re.compile(r"neg", re.I)


def _rows(path):
    with open(path, newline="") as f:
        return list(csv.DictReader(f))


def _name(r):
    n = r.get("Kernel_Name") or r.get("Kernel-Name") or r.get("KernelName") or ""
    return n.strip()


def _short(n):
    """The kernel's name without the return type and the argument list."""
    n = re.sub(r"^void ", "", n).replace("(anonymous namespace)", "{anonymous}")
    n = n.split("(")[0] if "(" in n and not n.startswith("(") else n
    return n.replace("{anonymous}", "(anonymous namespace)")


def _timed_slice(items, bench):
    dom = bench["roofline"]["kernel"]
    K = int(bench["steps"])
    L = int(bench["kernels_one_step"][dom]["launches"])
    after = (2 * K + 1) * L
    if len(items) < after + K * L:
        raise SystemExit("trace holds %d %s launches, fewer than the %d the bench sequence makes"
                         % (len(items), dom, after + K * L))
    return items[len(items) - after - K * L: len(items) - after]


def times(trace_csv, bench_json):
    bench = json.load(open(bench_json))
    rows = _rows(trace_csv)
    per = defaultdict(list)
    disp = []
    for r in rows:
        n = _short(_name(r))
        d = (int(r["End_Timestamp"]) - int(r["Start_Timestamp"])) / 1000.0
        per[n].append(d)
        disp.append((int(r["Start_Timestamp"]), n, d))
    disp.sort()
    tot = sum(sum(v) for v in per.values())
    print("| kernel | calls | total us | avg us | min us | max us | % |")
    print("|---|---|---|---|---|---|---|")
    for n, v in sorted(per.items(), key=lambda kv: -sum(kv[1])):
        print("| `%s` | %d | %.1f | %.2f | %.2f | %.2f | %.1f |"
              % (n[:100], len(v), sum(v), sum(v) / len(v), min(v), max(v), 100 * sum(v) / tot))
    dom = bench["roofline"]["kernel"]
    cls = [(n, d) for _, n, d in disp if CLASS_RE[dom].search(n)]
    sl = _timed_slice(cls, bench)
    avg = sum(d for _, d in sl) / len(sl)
    print()
    print("Timed region, class `%s`: %d launches, average %.2f us (rocprofv3); "
          "bench.py live HIP events: %.2f us over %d launches."
          % (dom, len(sl), avg, bench["roofline"]["avg_launch_ms"] * 1e3, bench["roofline"]["launches"]))
    names = sorted(set(n for n, _ in sl))
    print("Kernels of the class in the timed region: " + ", ".join("`%s`" % n for n in names))
    every = int(bench.get("event_every", 1))
    if every > 1:
        # the launches bench.py bracketed: those of steps 0, S, 2S, ...
        L = int(bench["kernels_one_step"][dom]["launches"])
        ev = [d for i, (_, d) in enumerate(sl) if (i // L) % every == 0]
        print("Launches of the bracketed steps (every %d-th): %d, average %.2f us (rocprofv3)."
              % (every, len(ev), sum(ev) / len(ev)))


def _counter(path, counter):
    out = []
    for r in _rows(path):
        if r.get("Counter_Name", counter) != counter:
            continue
        out.append((int(r.get("Dispatch_Id", r.get("Correlation_Id", 0))), _short(_name(r)),
                    float(r["Counter_Value"])))
    # one row per dispatch (values of the same dispatch summed over dimensions)
    agg = defaultdict(float)
    nm = {}
    for i, n, v in out:
        agg[i] += v
        nm[i] = n
    return [(i, nm[i], agg[i]) for i in sorted(agg)]


def traffic(fetch_csv, write_csv, bench_json, copy_mib):
    bench = json.load(open(bench_json))
    dom = bench["roofline"]["kernel"]
    copy_kib = float(copy_mib) * 1024.0
    res = {}
    for label, path, counter in (("fetch", fetch_csv, "FETCH_SIZE"), ("write", write_csv, "WRITE_SIZE")):
        rows = _counter(path, counter)
        cp = [v for _, n, v in rows if COPY_RE.search(n)]
        if not cp:
            raise SystemExit("no copy-probe dispatch in " + path)
        scale = copy_kib / max(cp)
        cls = [(n, v) for _, n, v in rows if CLASS_RE[dom].search(n)]
        sl = _timed_slice(cls, bench)
        kib = sum(v for _, v in sl) / len(sl)
        res[label] = {"counter": counter, "copy_probe_kib_measured": max(cp), "copy_probe_kib_expected": copy_kib,
                      "scale": scale, "kib_per_launch_raw": kib, "bytes_per_launch": kib * scale * 1024.0,
                      "launches": len(sl)}
    total = res["fetch"]["bytes_per_launch"] + res["write"]["bytes_per_launch"]
    alg = bench["roofline"]["algorithmic_bytes_per_launch"]
    prec = bench["config"].get("precision", "fp64")
    key = dom if prec == "fp64" else "%s@%s" % (dom, prec)
    print(json.dumps({key: {"kernel_digest": bench["kernel_digest"], "bytes_per_launch": total,
                            "algorithmic_bytes_per_launch": alg, "ratio_to_algorithmic": total / alg,
                            "fetch": res["fetch"], "write": res["write"],
                            "workload": bench["config"]["workload"]}}, indent=1))


def mfma(csv_path, bench_json):
    bench = json.load(open(bench_json))
    dom = bench["roofline"]["kernel"]
    per = defaultdict(dict)
    names = {}
    for r in _rows(csv_path):
        i = int(r.get("Dispatch_Id", r.get("Correlation_Id", 0)))
        per[i][r["Counter_Name"]] = per[i].get(r["Counter_Name"], 0.0) + float(r["Counter_Value"])
        names[i] = _short(_name(r))
    cls = [(names[i], per[i]) for i in sorted(per) if CLASS_RE[dom].search(names[i])]
    sl = _timed_slice(cls, bench)
    alg = bench["roofline"]["flops_per_launch"]
    out = {"launches": len(sl), "kernel_digest": bench["kernel_digest"], "workload": bench["config"]["workload"],
           "algorithmic_flops_per_launch": alg}
    for ty in ("F64", "F32", "BF16", "I8"):
        # each MOPS count stands for 512 operations of that type (int8: multiply-adds counted as two)
        cn = "SQ_INSTS_VALU_MFMA_MOPS_" + ty
        if any(cn in c for _, c in sl):
            mops = sum(c.get(cn, 0.0) for _, c in sl) / len(sl)
            out["mfma_flops_executed_per_launch"] = mops * 512.0
            out["mfma_type"] = ty
            # split bf16 runs three bf16 products per FP64-equivalent product
            out["executed_over_algorithmic"] = mops * 512.0 / alg
    if any("MfmaUtil" in c for _, c in sl):
        # rocprofv3's derived metric: MFMA busy cycles / (GPU active cycles x SIMDs), in percent
        out["mfma_util_percent_mean"] = sum(c["MfmaUtil"] for _, c in sl) / len(sl)
    # every counter of the pass, mean per launch, and the LDS / wait ratios when present
    keys = sorted({k for _, c in sl for k in c})
    out["counters_per_launch"] = {k: sum(c.get(k, 0.0) for _, c in sl) / len(sl) for k in keys}
    m = out["counters_per_launch"]
    if m.get("SQ_INSTS_LDS"):
        out["lds_bank_conflict_cycles_per_lds_instruction"] = m.get("SQ_LDS_BANK_CONFLICT", 0.0) / m["SQ_INSTS_LDS"]
    if m.get("SQ_WAVE_CYCLES"):
        for k in ("SQ_WAIT_INST_LDS", "SQ_WAIT_ANY"):
            if k in m:
                out[k.lower() + "_over_wave_cycles"] = m[k] / m["SQ_WAVE_CYCLES"]
    print(json.dumps({dom: out}, indent=1))


def timeline(trace_csv, index):
    rows = sorted(_rows(trace_csv), key=lambda r: int(r["Start_Timestamp"]))
    ups = [i for i, r in enumerate(rows) if re.search(r"(^|::)fetch_kernel", _name(r))]
    k = int(index)
    if k + 1 >= len(ups):
        raise SystemExit("only %d plan uploads in the trace" % len(ups))
    sel = rows[ups[k]:ups[k + 1] + 1]
    t0 = int(sel[0]["Start_Timestamp"])
    print("| start us | end us | us | queue | kernel |")
    print("|---|---|---|---|---|")
    spans = []
    for r in sel:
        s0, s1 = int(r["Start_Timestamp"]), int(r["End_Timestamp"])
        spans.append((s0, s1))
        print("| %.1f | %.1f | %.1f | %s | `%s` |" % ((s0 - t0) / 1e3, (s1 - t0) / 1e3, (s1 - s0) / 1e3,
                                                  r.get("Queue_Id", "?"), _short(_name(r))))
    spans.sort()
    busy, cur = 0, None
    for a, b in spans:
        if cur is None or a > cur[1]:
            if cur:
                busy += cur[1] - cur[0]
            cur = [a, b]
        else:
            cur[1] = max(cur[1], b)
    busy += cur[1] - cur[0]
    span = max(b for _, b in spans) - min(a for a, _ in spans)
    print()
    print("Window %.1f us: some kernel running %.1f us, idle %.1f us." % (span / 1e3, busy / 1e3, (span - busy) / 1e3))


STAGE_KIND = {0: "GEMM (1D exponentials)", 1: "Taylor sums", 2: "mode product, store",
              3: "last mode + node sum", 4: "last mode + squaring", 5: "mode product, store (64 x 128 tiles)",
              6: "last mode + node sum (8 waves)", 7: "last mode + squaring (8 waves)"}
BATCH_RE = re.compile(r"(^|::)batch(_wide)?_kernel<(\d+), (\d+), (true|false)>")


def batch(trace_csv):
    rows = sorted(_rows(trace_csv), key=lambda r: int(r["Start_Timestamp"]))
    runs, cur = [], []
    for r in rows:
        if BATCH_RE.search(_name(r)):
            cur.append(r)
        elif cur:
            runs.append(cur)
            cur = []
    if cur:
        runs.append(cur)
    if not runs:
        raise SystemExit("no batched-stage kernels in the trace")
    last = runs[-1]
    agg = defaultdict(lambda: [0, 0.0])
    for r in last:
        m = BATCH_RE.search(_name(r))
        key = (int(m.group(3)), int(m.group(4)), m.group(5))
        agg[key][0] += 1
        agg[key][1] += (int(r["End_Timestamp"]) - int(r["Start_Timestamp"])) / 1e6
    print("| stage kind | orders | 16-byte staging | launches | ms |")
    print("|---|---|---|---|---|")
    for (t, np_, vec), (n, ms) in sorted(agg.items()):
        print("| %s | %d | %s | %d | %.1f |" % (STAGE_KIND.get(t, str(t)), np_, vec, n, ms))
    total = sum(ms for _, ms in agg.values())
    span = (int(last[-1]["End_Timestamp"]) - int(last[0]["Start_Timestamp"])) / 1e6
    print()
    print("Sum of the last call: %.1f ms over %d launches, span %.1f ms." % (total, len(last), span))


if __name__ == "__main__":
    if len(sys.argv) >= 4 and sys.argv[1] == "times":
        times(sys.argv[2], sys.argv[3])
    elif len(sys.argv) >= 6 and sys.argv[1] == "traffic":
        traffic(sys.argv[2], sys.argv[3], sys.argv[4], sys.argv[5])
    elif len(sys.argv) >= 4 and sys.argv[1] == "mfma":
        mfma(sys.argv[2], sys.argv[3])
    elif len(sys.argv) >= 4 and sys.argv[1] == "timeline":
        timeline(sys.argv[2], sys.argv[3])
    elif len(sys.argv) >= 3 and sys.argv[1] == "batch":
        batch(sys.argv[2])
    else:
        print(__doc__)
        sys.exit(2)
