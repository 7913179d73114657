"""Kernel variants and graph replay.

* Every kernel variant (per-lane LDS list capacities) computes the same
  result bit for bit.
* A batch enqueue captured in a HIP graph (torch.cuda.CUDAGraph) replays
  correctly several times in a row, with eager library work and host
  synchronisations between the replays; every replay is checked against
  the eager result.
"""
from __future__ import annotations

import numpy as np
import pytest

from synth import gen
from tests.helpers import random_grid

pytestmark = pytest.mark.gpu


def _host(dg):
    cp, z = dg.to_host()
    return cp.copy(), z.astype(np.float64).copy()


def test_variants_identical(engine):
    import paper_1804_08968_amd as dx
    rng = np.random.default_rng(8)
    g = random_grid(rng, 150, 40, 80.0, max_per_col=6)
    dg = dx.DeviceGrid.from_host(g)
    try:
        ref = None
        for v in range(dx.NVARIANT):
            dx.dexel_set_variant(engine.ctx, v)
            for op, r in (("dilate", 4.5), ("close", 3.0)):
                print(f"[case] variant {v} {op}", flush=True)
                out = _host(engine.offset(dg, r, op))
                if ref is None:
                    ref = {}
                key = (op, r)
                if key in ref:
                    assert np.array_equal(out[0], ref[key][0]) and np.array_equal(out[1], ref[key][1])
                else:
                    ref[key] = out
    finally:
        dx.dexel_set_variant(engine.ctx, -1)


def test_graph_replay_batch(engine):
    import torch
    import paper_1804_08968_amd as dx
    shapes = gen.batch_shapes(2, count=5, smin=64, smax=160)
    dgs = [dx.DeviceGrid.from_host(g) for g, _ in shapes]
    radii = [r for _, r in shapes]
    ops = ["dilate", "close", "erode", "open", "dilate"]
    bp = dx.BatchPlan(engine, dgs, radii, ops)
    bp.enqueue(flags=dx.DEXEL_FLAG_SYNC)
    eager = [_host(g) for g in bp.results()]
    other = dx.Plan(engine, dgs[0], 2.0, "erode")
    s = torch.cuda.Stream()
    s.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(s):
        bp.enqueue()
    torch.cuda.synchronize()
    graph = torch.cuda.CUDAGraph()
    print("[case] capture", flush=True)
    with torch.cuda.graph(graph, stream=s):
        bp.enqueue(stream=s)
    torch.cuda.synchronize()
    for rep in range(4):
        for o in bp.outs:  # poison the outputs so a no-op replay would be caught
            o[0].fill_(-7)
            o[1].fill_(float("nan"))
        torch.cuda.synchronize()
        print(f"[case] replay {rep}", flush=True)
        graph.replay()
        torch.cuda.synchronize()
        assert bp.statuses() == [0] * len(dgs)
        got = [_host(g) for g in bp.results()]
        for a, b in zip(got, eager):
            assert np.array_equal(a[0], b[0]) and np.array_equal(a[1], b[1])
        other.enqueue(flags=dx.DEXEL_FLAG_SYNC)  # eager work between replays


def test_graph_replay_after_engine_workspace_grows(engine):
    """A captured plan keeps its own workspace: growing (and so reallocating)
    the engine's shared workspace after the capture leaves replays intact."""
    import torch
    import paper_1804_08968_amd as dx
    shapes = gen.batch_shapes(4, count=3, smin=64, smax=128)
    dgs = [dx.DeviceGrid.from_host(g) for g, _ in shapes]
    radii = [r for _, r in shapes]
    bp = dx.BatchPlan(engine, dgs, radii, ["close", "dilate", "erode"])
    bp.enqueue(flags=dx.DEXEL_FLAG_SYNC)
    eager = [_host(g) for g in bp.results()]
    s = torch.cuda.Stream()
    s.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(s):
        bp.enqueue()
    torch.cuda.synchronize()
    graph = torch.cuda.CUDAGraph()
    print("[case] capture", flush=True)
    with torch.cuda.graph(graph, stream=s):
        bp.enqueue(stream=s)
    torch.cuda.synchronize()
    big = dx.DeviceGrid.from_host(gen.primitives_grid(3, n=256, count=400))
    for rep in range(3):
        have = engine.workspace(1).numel()
        engine.workspace(have + (64 << 20))      # frees the old buffer, allocates a larger one
        engine.offset(big, 6.0 + rep, "close")   # eager work in the reallocated workspace
        for o in bp.outs:
            o[0].fill_(-7)
            o[1].fill_(float("nan"))
        torch.cuda.synchronize()
        print(f"[case] replay {rep} after growing the engine workspace", flush=True)
        graph.replay()
        torch.cuda.synchronize()
        assert bp.statuses() == [0] * len(dgs)
        for a, b in zip((_host(g) for g in bp.results()), eager):
            assert np.array_equal(a[0], b[0]) and np.array_equal(a[1], b[1])
