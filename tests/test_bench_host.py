"""Host-side parts of bench.py (no GPU): the one-GPU guard, the CPU baseline
record and the kernel-source digest that keys the committed HBM counters."""
import json
import os
import subprocess
import sys

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)

import bench  # noqa: E402
from paper_2211_00696_amd import inputs as I  # noqa: E402


def test_more_than_one_gpu_is_refused():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"], capture_output=True,
                       text=True, timeout=120, cwd=ROOT)
    assert r.returncode == 2
    msg = json.loads(r.stdout.strip().splitlines()[-1])
    assert "one GPU" in msg["error"]


def test_cpu_baseline_record():
    pr = I.problem("advdiff3d", seed=0, n=8)
    out = np.zeros((pr["p"] + 1, pr["v"].size))
    cb, errs = bench.cpu_baseline(pr, out, min_seconds=0.05, max_runs=3)
    assert cb["kind"] == "oracle" and cb["unit"] == "grid-pts/s"
    assert 1 <= len(cb["run_seconds"]) <= 3
    assert cb["value"] == pr["v"].size / float(np.median(cb["run_seconds"]))
    assert cb["cores"] >= 1 and cb["affinity_cores"] >= 1
    assert cb["cpu_model"] is None or isinstance(cb["cpu_model"], str)
    # out is all zeros: every phi_k differs from the oracle by 100%
    assert len(errs) == pr["p"] + 1 and all(abs(e - 1.0) < 1e-12 for e in errs)


def test_kernel_digest_covers_every_kernel_source():
    csrc = os.path.join(ROOT, "paper_2211_00696_amd", "csrc")
    kernels = sorted(f for f in os.listdir(csrc) if f.startswith(("kernels", "tile_")))
    src = open(os.path.join(ROOT, "bench.py")).read()
    for f in kernels:
        assert '"%s"' % f in src, f
    assert len(bench.kernel_source_digest()) == 16


def test_traffic_entries_are_current_and_tied_to_their_workload():
    """The bench line uses a committed counter entry only for the kernel sources and the workload it
    was measured on: the headline problem at n = 256 (FP64, FP32, split bf16) and the int8 digits at
    n = 128, not the same form at another size or rule, nor after a kernel source changed."""
    d = json.load(open(os.path.join(ROOT, "profiles", "traffic.json")))
    where = {"ttm_store": (256, "fp64"), "ttm_store@fp32": (256, "fp32"), "ttm_store@bf16x3": (256, "bf16x3"),
             "ttm_store@int8": (128, "int8")}
    assert set(d) == set(where)
    for key, (n, prec) in where.items():
        digest = d[key]["kernel_digest"]
        wl = bench.headline_workload(n, n ** 3, 0, "gauss", prec)
        assert bench.load_traffic("ttm_store", digest, prec, wl) == d[key]["bytes_per_launch"]
        other = 128 if n == 256 else 256
        assert bench.load_traffic("ttm_store", digest, prec, bench.headline_workload(other, other ** 3, 0, "gauss", prec)) is None
        assert bench.load_traffic("ttm_store", digest, prec, bench.headline_workload(n, n ** 3, 0, "cc", prec)) is None
        assert bench.load_traffic("ttm_store", "0" * 16, prec, wl) is None
