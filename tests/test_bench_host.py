"""Host-side pieces of bench.py: the algorithmic byte count, the stored
traffic lookup, and the one-GPU guard (no GPU needed)."""
from __future__ import annotations

import json
import os
import subprocess
import sys

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)

import bench  # noqa: E402


def test_algorithmic_bytes_counts_each_term():
    """Graph part: |V|*d*s + hops*R*4 + d*4; leaf scan: w*d*4 + d*4; rerank:
    min(m, |V|, width)*d*4 per graph part; outputs k*12 per query."""
    d, R, k = 8, 4, 3
    tr = {"kind": np.array([[1, 2], [1, 0]]), "n_visited": np.array([[10, 5], [50, 0]]),
          "hops": np.array([[2, 0], [7, 0]]), "x": np.array([[0, 0], [0, 0]]),
          "y": np.array([[99, 4], [19, 0]])}
    m = np.array([[6, 6], [30, 30]])
    plain = bench.algorithmic_bytes(tr, d, R, k, m, 4.0, False)
    graph = (10 + 50) * d * 4 + (2 + 7) * R * 4 + 2 * d * 4
    scan = 5 * d * 4 + d * 4
    out = 2 * k * 12
    assert plain == graph + scan + out
    rer = bench.algorithmic_bytes(tr, d, R, k, m, 2.0, True)
    graph16 = (10 + 50) * d * 2 + (2 + 7) * R * 4 + 2 * d * 4
    assert rer == graph16 + scan + out + (min(6, 10, 100) + min(30, 50, 20)) * d * 4


def test_stored_traffic_needs_matching_key_and_sources():
    key = {"workload": "none", "nq": -1}
    assert bench.stored_traffic(key) is None
    sha = bench.kernel_sources_sha256()
    assert len(sha) == 64 and sha == bench.kernel_sources_sha256()
    for f in os.listdir(os.path.join(ROOT, "profiles")):
        for line in open(os.path.join(ROOT, "profiles", f)):
            if line.startswith("traffic-record: "):
                rec = json.loads(line[len("traffic-record: "):])
                assert rec["hbm_bytes_per_launch"] > 0 and len(rec["sources_sha256"]) == 64


def test_more_than_one_gpu_is_refused():
    p = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"],
                       capture_output=True, text=True, timeout=120)
    assert p.returncode == 2
    assert "one GPU" in json.loads(p.stdout.strip().splitlines()[-1])["error"]
