"""Host logic of bench.py (CPU): the candidate-pair count behind the
dexelisation roofline, the staleness guard of the measured HBM traffic, and
the refusal of more than one GPU."""
from __future__ import annotations

import math
import os
import subprocess
import sys

import numpy as np
import pytest

import bench

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


@pytest.mark.parametrize("seed", range(3))
def test_candidate_pairs_brute_force(seed):
    """Every (cell, primitive) pair whose cell index lies in the primitive's
    clipped cell bounding box, counted cell by cell."""
    rng = np.random.default_rng(seed)
    n = 23
    rec = []
    for _ in range(30):
        if rng.random() < 0.5:
            rec.append((0.0, *rng.uniform(-5, n + 5, 3), rng.uniform(0.2, 6.0), 0.0, 0.0))
        else:
            lo = rng.uniform(-5, n + 5, 3)
            rec.append((1.0, *lo, *(lo + rng.uniform(0.0, 9.0, 3))))
    want = 0
    for p in rec:
        if p[0] == 0.0:
            lo, hi = (p[1] - p[4], p[2] - p[4]), (p[1] + p[4], p[2] + p[4])
        else:
            lo, hi = (p[1], p[2]), (p[4], p[5])
        for y in range(n):
            for x in range(n):
                if math.ceil(lo[0] - 0.5) <= x <= math.floor(hi[0] - 0.5) and \
                        math.ceil(lo[1] - 0.5) <= y <= math.floor(hi[1] - 0.5):
                    want += 1
    assert bench.dex_candidate_pairs(np.asarray(rec), n) == want


def test_traffic_only_for_the_profiled_source(monkeypatch):
    """The committed traffic summary is used only while its source hash is the
    kernels' own; any other source reads as unmeasured."""
    real = bench.measured_traffic("k_union")
    assert real is not None and real > 0
    monkeypatch.setattr(bench, "kernels_sha256", lambda: "0" * 64)
    assert bench.measured_traffic("k_union") is None


def test_more_than_one_gpu_is_refused():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"],
                       capture_output=True, text=True, timeout=120, cwd=ROOT)
    assert r.returncode == 2
    assert "one GPU" in r.stderr
