"""Parity at full benchmark size: the closing (r = 16) of the 2048 x 2048
gyroid lattice (2.15e8 intervals), run as bench.py runs it (a Plan with the
autotuned kernel variant), checked on sampled output columns against the
oracle evaluated on just those columns.

The samples include the grid corners and the x-border columns, which take
the heavy-column (z-slab) replays, and columns next to them.
"""
from __future__ import annotations

import numpy as np
import pytest

from synth import gen
from tests.helpers import compare_columns

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def c3_grid():
    return gen.gyroid_grid(0)


def sample_columns(n, seed=3, count=24):
    pts = [(0, 0), (n - 1, 0), (0, n - 1), (n - 1, n - 1), (0, 1000), (1, 1000), (2, 1000),
           (3, 1001), (n - 1, 1000), (n - 2, 777), (n - 3, 778), (1000, 0), (1000, 1),
           (1000, n - 1), (1000, n - 2), (3, 5)]
    rng = np.random.default_rng(seed)
    pts += [tuple(int(v) for v in p) for p in rng.integers(0, n, size=(count, 2))]
    return np.unique(np.array([y * n + x for x, y in pts], np.int64))


@pytest.mark.parametrize("op", ["close"])
def test_c3_closing_sampled(engine, oracle_lib, c3_grid, op):
    import paper_1804_08968_amd as dx
    g = c3_grid
    print(f"[case] c3 {op} r=16 {g.nx}x{g.ny} nseg={g.nseg}", flush=True)
    dg = dx.DeviceGrid.from_host(g)
    plan = dx.Plan(engine, dg, 16.0, op)
    chosen, _ = plan.autotune(reps=1)
    plan.enqueue(flags=dx.DEXEL_FLAG_SYNC)
    assert plan.status() == dx.DEXEL_OK
    col_ptr, z = plan.result().to_host()
    cols = sample_columns(g.nx)
    gcnt = np.diff(col_ptr)[cols]
    gz = np.concatenate([z[2 * col_ptr[c]: 2 * col_ptr[c + 1]] for c in cols]).astype(np.float64)
    c32, z32 = oracle_lib.region_chain(g, 16.0, op, cols, "f32model")
    assert np.array_equal(gcnt, c32), f"variant {chosen}: counts differ from the float32 model"
    assert np.array_equal(gz, z32), f"variant {chosen}: endpoints differ from the float32 model"
    c64, z64 = oracle_lib.region_chain(g, 16.0, op, cols, "f64")
    res = compare_columns(c64, z64, gcnt, gz, 16.0, k=2)
    assert res["failed"] == 0, res
    # every column of the output is canonical
    assert col_ptr[0] == 0 and np.all(np.diff(col_ptr) >= 0)
    zz = z[: 2 * col_ptr[-1]].reshape(-1, 2)
    assert np.all(zz[:, 0] <= zz[:, 1])
