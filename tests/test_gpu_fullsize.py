"""Parity at full benchmark size on the 2048 x 2048 gyroid lattice (2.15e8
intervals, about 51 per column), against the oracle evaluated on whole
64 x 64 tiles of output columns.

* The closing at r = 16, run as bench.py runs it (a Plan with the autotuned
  kernel variant).  Its dilation fills the lattice, so the closing keeps
  about one interval per column.
* The same grid dilated at r = 4 and r = 8 and eroded at r = 1 and r = 2.
  There the output keeps many intervals per column (about 47, 35 and 52;
  the r = 2 erosion removes most walls), so the seed, neighbour and union
  paths and the heavy-column (z-slab) replays at the grid's x borders all
  decide the result.

Eight tiles per case: the four grid corners, the middles of both x borders,
the centre and one seeded random tile.  Each is compared bit for bit with
the oracle's float32 model and within tolerance with its float64 result
(the brute force of Sec. 4, "Baseline Comparison").
"""
from __future__ import annotations

import numpy as np
import pytest

from synth import gen
from tests.helpers import compare_columns

pytestmark = pytest.mark.gpu

N = 2048
T = 64


def tile_origins(n=N, seed=5):
    rng = np.random.default_rng(seed)
    m = n // 2 - T // 2
    rx, ry = (int(v) for v in rng.integers(0, n - T, 2))
    return [("corner00", 0, 0), ("corner10", n - T, 0), ("corner01", 0, n - T),
            ("corner11", n - T, n - T), ("xborder0", 0, m), ("xborder1", n - T, m),
            ("centre", m, m), ("random", rx, ry)]


TILES = tile_origins()


def tile_cols(x0, y0, n=N):
    return (np.arange(y0, y0 + T)[:, None] * n + np.arange(x0, x0 + T)[None, :]).ravel().astype(np.int64)


@pytest.fixture(scope="module")
def c3_grid():
    return gen.gyroid_grid(0)


def _gpu(engine, g, r, op, autotune):
    import paper_1804_08968_amd as dx
    print(f"[case] gyroid2048 {op} r={r} (GPU)", flush=True)
    dg = dx.DeviceGrid.from_host(g)
    if autotune:
        plan = dx.Plan(engine, dg, r, op)
        plan.autotune(reps=1)
        plan.enqueue(flags=dx.DEXEL_FLAG_SYNC)
        assert plan.status() == dx.DEXEL_OK
        col_ptr, z = plan.result().to_host()
    else:
        col_ptr, z = engine.offset(dg, r, op).to_host()
    assert col_ptr[0] == 0 and np.all(np.diff(col_ptr) >= 0)
    zz = z[: 2 * col_ptr[-1]].reshape(-1, 2)
    assert np.all(zz[:, 0] <= zz[:, 1])
    return col_ptr, z


@pytest.fixture(scope="module")
def results():
    return {}


def _result(results, engine, g, r, op):
    key = (r, op)
    if key not in results:
        results.clear()  # one 2048^2 result on the host at a time
        results[key] = _gpu(engine, g, r, op, autotune=(op == "close"))
    return results[key]


def _check_tile(oracle, g, r, op, col_ptr, z, x0, y0, name):
    cols = tile_cols(x0, y0)
    print(f"[case] gyroid2048 {op} r={r} tile {name} ({x0}, {y0}) (oracle)", flush=True)
    gcnt = np.diff(col_ptr)[cols]
    gz = np.concatenate([z[2 * col_ptr[c]: 2 * col_ptr[c + 1]] for c in cols]).astype(np.float64)
    if op in ("dilate", "erode"):
        c32, z32 = oracle.offset_columns(g, r, op, "f32model", cols=cols)
        c64, z64 = oracle.offset_columns(g, r, op, "f64", cols=cols)
    else:
        c32, z32 = oracle.region_chain(g, r, op, cols, "f32model")
        c64, z64 = oracle.region_chain(g, r, op, cols, "f64")
    assert np.array_equal(gcnt, c32), f"{name}: counts differ from the float32 model"
    assert np.array_equal(gz, z32), f"{name}: endpoints differ from the float32 model"
    res = compare_columns(c64, z64, gcnt, gz, r, k=2 if op in ("open", "close") else 1)
    assert res["failed"] == 0, (name, res)
    return gcnt


@pytest.mark.parametrize("name,x0,y0", TILES)
def test_c3_closing_tiles(engine, oracle_lib, c3_grid, results, name, x0, y0):
    col_ptr, z = _result(results, engine, c3_grid, 16.0, "close")
    _check_tile(oracle_lib, c3_grid, 16.0, "close", col_ptr, z, x0, y0, name)


def test_c3_closing_thin_equals_general(engine, c3_grid, results):
    """The whole 2048^2 closing: the erosion pass's thin-column filter (the
    bench's path) gives the same grid, bit for bit, as the general kernels."""
    import paper_1804_08968_amd as dx
    col_ptr, z = _result(results, engine, c3_grid, 16.0, "close")
    print("[case] gyroid2048 close r=16 general kernels (GPU)", flush=True)
    dg = dx.DeviceGrid.from_host(c3_grid)
    gcp, gz = engine.offset(dg, 16.0, "close", flags=dx.DEXEL_FLAG_GENERAL).to_host()
    assert np.array_equal(col_ptr, gcp)
    assert np.array_equal(z[: 2 * col_ptr[-1]], gz[: 2 * gcp[-1]])


@pytest.mark.parametrize("name,x0,y0", TILES)
@pytest.mark.parametrize("op,r", [("dilate", 4.0), ("dilate", 8.0), ("erode", 1.0), ("erode", 2.0)])
def test_gyroid2048_fragmented_tiles(engine, oracle_lib, c3_grid, results, op, r, name, x0, y0):
    col_ptr, z = _result(results, engine, c3_grid, r, op)
    gcnt = _check_tile(oracle_lib, c3_grid, r, op, col_ptr, z, x0, y0, name)
    if (op, r) != ("erode", 2.0):
        # the output really is fragmented (tens of intervals per column)
        assert gcnt.mean() > 10.0, (name, gcnt.mean())
