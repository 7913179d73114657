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


def test_traffic_only_for_the_profiled_source(monkeypatch, tmp_path):
    """A traffic summary is used only while its source hash is the kernels'
    own; any other source reads as unmeasured.  Each counter is scaled by
    what it read for the copy of known size."""
    f = tmp_path / "traffic.txt"
    f.write_text("# summary\n"
                 f"kernels_source_sha256 {bench.kernels_sha256()}\n"
                 "copy_bytes 1073741824\ncopy_fetch_kib 524288\ncopy_write_kib 1048576\n"
                 "kernel k_union 1000 300   # comment\n")
    monkeypatch.setattr(bench, "TRAFFIC_FILE", str(f))
    assert bench.measured_traffic("k_union") == (1000 * 2.0 + 300 * 1.0) * 1024
    assert bench.measured_traffic("k_seeds") is None
    monkeypatch.setattr(bench, "kernels_sha256", lambda: "0" * 64)
    assert bench.measured_traffic("k_union") is None


class _Dx:
    PROFILE_STAGES = ["column_gaps", "direct", "thin_erosion", "chord_extremes", "row_offset", "row_offset_replay",
                      "gap_cut", "neighbour", "neighbour_replay", "seeds", "seeds_replay", "y_union",
                      "y_union_replay", "result_scan", "compact"]
    PROFILE_KERNELS = ["k_col_gaps", "k_direct", "k_thin_erode", "k_solid_dilate", "k_row_offset", "k_row_offset_fb",
                       "k_gap_cut", "k_neighbour", "k_neighbour_fb", "k_seeds", "k_seeds_fb", "k_union",
                       "k_union_fb", "k_scan", "k_copy_out"]


def test_dominant_stage_counts_its_replay():
    """The dominant stage is the costliest by main plus replay time; the
    reported kernel is the launch group carrying >= 90% of it, or both."""
    st = {"row_offset": 100, "neighbour": 100, "seeds": 1000, "result": 100}
    b = bench.kernel_bytes("row_offset", 64, 500, st)
    per = {k: 0.0 for k in _Dx.PROFILE_STAGES}
    per.update(row_offset=2.0, row_offset_replay=6.0, y_union=5.0, y_union_replay=0.5)
    roof = bench.stage_roofline(_Dx, per, [(500, st), (500, st)], 64)
    assert roof["stage"] == "row_offset" and roof["kernel"] == "k_row_offset + k_row_offset_fb"
    assert roof["kernel_ms"] == 4.0 and roof["stage_ms"] == 4.0
    assert roof["bytes_per_launch"] == b
    assert abs(roof["frac"] - b / 4e-3 / 1e9 / bench.HBM_PEAK_GBS) < 1e-5
    assert abs(roof["stage_frac"] - roof["frac"]) < 1e-5
    # the replay does the stage's work: it is the kernel
    per.update(row_offset=0.2, row_offset_replay=7.8)
    roof = bench.stage_roofline(_Dx, per, [(500, st), (500, st)], 64)
    assert roof["kernel"] == "k_row_offset_fb" and roof["kernel_ms"] == 3.9
    assert abs(roof["frac"] - b / 3.9e-3 / 1e9 / bench.HBM_PEAK_GBS) < 1e-5
    assert abs(roof["stage_frac"] - b / 4e-3 / 1e9 / bench.HBM_PEAK_GBS) < 1e-5
    # the main kernel does it
    per.update(row_offset=7.8, row_offset_replay=0.2)
    roof = bench.stage_roofline(_Dx, per, [(500, st), (500, st)], 64)
    assert roof["kernel"] == "k_row_offset" and roof["kernel_ms"] == 3.9


def test_step_bytes():
    """B_alg and B_min of a pass from the sizes it reports."""
    st = {"row_offset": 0, "neighbour": 0, "seeds": 7, "result": 3}
    alg, mn = bench.pass_bytes(10, 5, st)
    ptr = 8 * 11
    assert mn == ptr + 8 * 5 + ptr + 8 * 3
    assert alg == mn + 2 * (ptr + 9 * 7)
    r = bench.step_roofline([(5, st), (3, st)], 10, 1.0)
    assert r["step_bytes_min"] == mn + bench.pass_bytes(10, 3, st)[1]


def test_more_than_one_gpu_is_refused():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"],
                       capture_output=True, text=True, timeout=120, cwd=ROOT)
    assert r.returncode == 2
    assert "one GPU" in r.stderr
