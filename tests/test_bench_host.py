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
