"""The rocprofv3 summaries (host only) on synthetic trace and counter files
laid out as bench.py's step sequence: K timed calls, K unbracketed calls,
one plan execution and K executions of a reused plan, each making L launches
of the dominant class.  Durations and counter values encode each launch's
position, so picking the wrong launches changes the printed figures."""
import csv
import json
import os
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)

from paper_2211_00696_amd import rocprof_summary as R  # noqa: E402

K, L = 4, 3
STORE = "void phiq::ttm_store_kernel<phiq::Tile<64, 128, 16, 2, 4, 1, 1>, true, false>(phiq::TtmArgs)"
OTHER = "void phiq::gemm_panel_kernel(phiq::GemmJob const*)"


def launches():
    """(name, position among the class's launches or -1) in dispatch order:
    one warm-up call, then the bench sequence; a GEMM between stores."""
    seq = []
    calls = 1 + K + K + 1 + K
    for c in range(calls):
        for j in range(L):
            seq.append((OTHER, -1))
            seq.append((STORE, c * L + j))
    return seq


def bench_json(tmp_path, every=1):
    b = {"steps": K, "roofline": {"kernel": "ttm_store", "avg_launch_ms": 0.05, "launches": K * L,
                                  "algorithmic_bytes_per_launch": 1000.0, "flops_per_launch": 1e6},
         "kernels_one_step": {"ttm_store": {"launches": L}}, "event_every": every,
         "kernel_digest": "0123456789abcdef", "config": {"workload": "synthetic"}}
    p = tmp_path / "bench.json"
    p.write_text(json.dumps(b))
    return str(p)


def write_trace(tmp_path):
    p = tmp_path / "trace.csv"
    with open(p, "w", newline="") as f:
        w = csv.writer(f)
        w.writerow(["Kernel_Name", "Start_Timestamp", "End_Timestamp", "Queue_Id"])
        t = 0
        for name, pos in launches():
            d = 1000 * (pos + 1) if pos >= 0 else 500  # ns: position + 1 microseconds
            w.writerow([name, t, t + d, 1])
            t += d + 100
    return str(p)


def timed_positions():
    # the K timed calls follow the warm-up call
    return list(range(L, L + K * L))


def test_class_patterns():
    assert R.CLASS_RE["ttm_store"].search(R._short(STORE))
    assert R.CLASS_RE["gemm"].search(R._short(OTHER))
    assert R.CLASS_RE["gemm"].search("phiq::gemm_jobs_kernel<phiq::Tile<32, 32, 16, 1, 1, 2, 1> >")
    assert not R.CLASS_RE["ttm_store"].search("phiq::ttm_square_all_kernel<x>")


def test_times_takes_the_timed_calls(tmp_path, capsys):
    R.times(write_trace(tmp_path), bench_json(tmp_path))
    out = capsys.readouterr().out
    want = sum(p + 1 for p in timed_positions()) / len(timed_positions())
    assert "Timed region, class `ttm_store`: %d launches, average %.2f us" % (K * L, want) in out
    assert "Launches of the bracketed steps" not in out


def test_times_bracketed_steps(tmp_path, capsys):
    every = 2
    R.times(write_trace(tmp_path), bench_json(tmp_path, every))
    out = capsys.readouterr().out
    pos = [p for i, p in enumerate(timed_positions()) if (i // L) % every == 0]
    assert "every %d-th): %d, average %.2f us" % (every, len(pos), sum(p + 1 for p in pos) / len(pos)) in out


def write_counters(tmp_path, counter, copy_kib):
    p = tmp_path / (counter + ".csv")
    with open(p, "w", newline="") as f:
        w = csv.writer(f)
        w.writerow(["Dispatch_Id", "Kernel_Name", "Counter_Name", "Counter_Value"])
        did = 0
        # the copy probe first, split over two dimensions of one dispatch
        w.writerow([did, "at::native::vectorized_elementwise_kernel<4, at::native::neg_kernel_cuda>", counter,
                    copy_kib / 2])
        w.writerow([did, "at::native::vectorized_elementwise_kernel<4, at::native::neg_kernel_cuda>", counter,
                    copy_kib / 2])
        for name, pos in launches():
            did += 1
            w.writerow([did, name, counter, 10.0 * (pos + 1) if pos >= 0 else 7.0])
    return str(p)


def test_traffic_scales_by_the_copy_probe(tmp_path, capsys):
    copy_mib = 4
    # FETCH reads half the probe's bytes (scale 2), WRITE all of them (scale 1)
    f = write_counters(tmp_path, "FETCH_SIZE", copy_mib * 1024 / 2)
    w = write_counters(tmp_path, "WRITE_SIZE", copy_mib * 1024)
    R.traffic(f, w, bench_json(tmp_path), copy_mib)
    res = json.loads(capsys.readouterr().out)["ttm_store"]
    kib = sum(10.0 * (p + 1) for p in timed_positions()) / len(timed_positions())
    assert res["fetch"]["scale"] == pytest.approx(2.0)
    assert res["write"]["scale"] == pytest.approx(1.0)
    assert res["fetch"]["kib_per_launch_raw"] == pytest.approx(kib)
    assert res["bytes_per_launch"] == pytest.approx(kib * 1024 * 3.0)
    assert res["ratio_to_algorithmic"] == pytest.approx(kib * 1024 * 3.0 / 1000.0)
    assert res["kernel_digest"] == "0123456789abcdef"
