"""Direct evaluation of fragmented passes: each output column as the union of
its stencil's chords (Sec. 4, "Baseline Comparison"), by teams of lanes.

The library evaluates a pass directly when its input holds many intervals
per column and the stencil is small (at least 6 items per column, R <= 16,
at most 24000 chords per output column); the result is the definition
itself, so it must equal the staged kernels' result bit for bit.  Each case
is checked against the oracle's float32 model (bit-exact), the float64
oracle (tolerance) and the same call with DEXEL_FLAG_GENERAL (bit-exact).

Cases: columns of many thin intervals at radii 0 .. 6 on grids cut raggedly
by the teams, dilation, erosion and both chains; gyroid crops; a column of
thousands of separate intervals whose slabs overflow the team lists (the
whole-wave evaluation) and then the whole-wave lists (the arena tier);
empty columns and rows; and a batch mixing directly evaluated shapes with
staged ones.
"""
from __future__ import annotations

import numpy as np
import pytest

from synth import gen
from tests.helpers import grid_from_columns
from tests.test_gpu_thin import _rng, check, slab_grid, thin_grid

pytestmark = pytest.mark.gpu


def frag_grid(rng, nx, ny, kmin, kmax, height, p_empty=0.0):
    """kmin..kmax disjoint short intervals per column at random heights."""
    cols = []
    for _ in range(nx * ny):
        if rng.random() < p_empty:
            cols.append([])
            continue
        k = int(rng.integers(kmin, kmax + 1))
        pts = np.sort(rng.uniform(0, height, size=2 * k)).astype(np.float32).astype(np.float64)
        iv = []
        for i in range(k):
            a, b = pts[2 * i], pts[2 * i + 1]
            if iv and a <= iv[-1][1]:
                iv[-1] = (iv[-1][0], max(b, iv[-1][1]))
            else:
                iv.append((a, b))
        cols.append(iv)
    return grid_from_columns(nx, ny, cols)


@pytest.mark.parametrize("nx,ny", [(1, 1), (1, 40), (70, 1), (17, 9), (65, 33)])
@pytest.mark.parametrize("r", [0.0, 1.5, 4.0])
@pytest.mark.parametrize("op", ["dilate", "erode"])
def test_direct_sizes(engine, oracle_lib, nx, ny, r, op):
    g = frag_grid(_rng("direct-sizes", nx, ny, r, op), nx, ny, 6, 20, 400.0, p_empty=0.05)
    check(engine, oracle_lib, g, r, op, "direct sizes")


@pytest.mark.parametrize("r", [0.5, 2.0, 3.5, 6.0])
@pytest.mark.parametrize("op", ["dilate", "erode", "close", "open"])
def test_direct_radii(engine, oracle_lib, r, op):
    g = frag_grid(_rng("direct-radii", r, op), 48, 40, 8, 40, 800.0, p_empty=0.02)
    check(engine, oracle_lib, g, r, op, "direct radii")


@pytest.mark.parametrize("r", [1.0, 2.5, 5.0])
@pytest.mark.parametrize("op", ["dilate", "erode"])
def test_direct_gyroid_crop(engine, oracle_lib, r, op):
    g = gen.gyroid_grid(2, n=80, height=240.0, period=20.0)
    assert g.nseg >= 6 * g.nx * g.ny
    check(engine, oracle_lib, g, r, op, "direct gyroid80")


def _dense_column_grid(nx, ny, c0, count, spacing, length, top):
    """Every column one interval [0, top] but column c0, which holds `count`
    separate intervals [i * spacing, i * spacing + length]."""
    cols = [[(0.0, top)] for _ in range(nx * ny)]
    cols[c0] = [(float(np.float32(i * spacing)), float(np.float32(i * spacing + length)))
                for i in range(count)]
    return grid_from_columns(nx, ny, cols)


@pytest.mark.parametrize("n,count,spread,tier", [(5, 200, 25.0, "wave"), (20, 3000, 1.0, "arena")])
@pytest.mark.parametrize("op", ["dilate", "erode"])
def test_direct_overflow_tiers(engine, oracle_lib, n, count, spread, tier, op):
    """A column of `count` separate intervals among columns [0, 5000]: its
    team's four slab lists (24 each) overflow.  Spread over the whole range
    (200, 25 apart) they fit the whole wave's 64 slabs of 32; packed (3000,
    1 or 2 apart) they overflow those too and go to the arena tier."""
    nx = ny = n
    # chords 0.625 long (dilation at r = 0.25 of intervals 0.125 long);
    # gaps of the erosion's complement 1.0 long, 1.5 with their chord
    spacing, length = (spread, 0.125) if op == "dilate" else (2.0 * spread, 1.0)
    g = _dense_column_grid(nx, ny, (n // 2) * nx + n // 2, count, spacing, length, 5000.0)
    assert g.nseg >= 6 * nx * ny  # fragmented enough for the direct evaluation
    cp = check(engine, oracle_lib, g, 0.25, op, f"direct overflow {tier}")
    assert np.diff(cp)[(n // 2) * nx + n // 2] == count  # the intervals stay apart


def test_direct_empty_rows(engine, oracle_lib):
    rng = _rng("direct-empty")
    g = frag_grid(rng, 30, 24, 8, 16, 300.0)
    cols = [list(zip(g.z[2 * g.col_ptr[c]: 2 * g.col_ptr[c + 1]: 2],
                     g.z[2 * g.col_ptr[c] + 1: 2 * g.col_ptr[c + 1]: 2])) for c in range(g.nx * g.ny)]
    for x in range(30):
        cols[7 * 30 + x] = []
    for y in range(24):
        cols[y * 30 + 4] = []
    g2 = grid_from_columns(30, 24, cols)
    for op in ("dilate", "erode"):
        check(engine, oracle_lib, g2, 2.0, op, f"direct empty rows {op}")


def test_direct_in_batch(engine, oracle_lib):
    """Directly evaluated shapes among staged and tiled ones in one batch."""
    import paper_1804_08968_amd as dx
    rng = _rng("direct-batch")
    grids = [frag_grid(rng, 40, 30, 8, 20, 300.0), slab_grid(rng, 70, 20, 0.0, 30.0, 3.0),
             frag_grid(rng, 33, 65, 6, 12, 200.0), thin_grid(rng, 64, 64, 30.0, p_thick=0.1),
             frag_grid(rng, 1, 1, 10, 10, 50.0), gen.gyroid_grid(3, n=48, height=120.0, period=16.0)]
    radii = [2.0, 3.5, 1.0, 4.0, 0.0, 3.0]
    ops = ["dilate", "close", "erode", "open", "dilate", "open"]
    dgs = [dx.DeviceGrid.from_host(g) for g in grids]
    print("[case] direct batch", flush=True)
    outs = dx.batch_offset(engine, dgs, radii, ops)
    for g, r, op, o in zip(grids, radii, ops, outs):
        col_ptr, z = o.to_host()
        ref = oracle_lib.run(g, r, op, "f32model")
        assert np.array_equal(col_ptr, ref.col_ptr), (op, r)
        assert np.array_equal(z[: 2 * col_ptr[-1]].astype(np.float64), ref.z), (op, r)
