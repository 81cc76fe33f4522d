"""The benchmark's contract on the host: one GPU only, and its byte
accounting."""
import os
import subprocess
import sys

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)
import bench  # noqa: E402
from paper_0912_4273_amd import gridgen as G  # noqa: E402


def test_more_than_one_gpu_is_refused():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"],
                       capture_output=True, text=True, timeout=120)
    assert r.returncode == 2
    assert "one GPU" in r.stderr
    assert r.stdout == ""


def test_algorithmic_bytes():
    # read + write of an fp32 word, 2 B of routing, 110 B per vertex over 84 bins
    assert abs(bench.algorithmic_bytes_per_update(84, 4) - (8 + 2 + 110 / 84)) < 1e-12
    w = G.small_random(200, seed=3, n_bins=21)
    all_dct = bench.combined_bytes_per_step(w, np.zeros(w.n, np.int8), 4)
    assert abs(all_dct - w.n * w.k * bench.algorithmic_bytes_per_update(w.k, 4)) < 1e-6
    all_bal = bench.combined_bytes_per_step(w, np.ones(w.n, np.int8), 4)
    assert abs(all_bal - (w.n_edges * 9.0 + 110.0 * w.n)) < 1e-6


def test_traffic_only_for_the_profiled_kernel_source(monkeypatch):
    """`roofline.traffic` quotes the committed counter summary only while it
    was taken on the current kernel source; any other source gives null."""
    import json
    d = json.load(open(os.path.join(ROOT, "profiles", "sweep_traffic.json")))
    key = "stromgren_262144_k84_1000sweeps"
    e = d[key]
    assert abs(e["bytes_per_launch"] - (e["fetch_bytes"] + e["write_bytes"])) <= 2
    assert e["bytes_per_launch"] >= e["algorithmic_bytes"]
    monkeypatch.setattr(bench, "kernel_source_hash", lambda: e["kernel_sha"])
    assert bench.measured_traffic(key) == e["bytes_per_launch"]
    assert bench.measured_traffic("no_such_workload") is None
    monkeypatch.setattr(bench, "kernel_source_hash", lambda: "0" * 16)
    assert bench.measured_traffic(key) is None
