"""Dilation of columns whose result is one interval: the tiled test against
the oracle and against the general kernels.

Every chord of a column's stencil lies in [L, U], L the smallest chord start
and U the largest chord end (Sec. 4, "Baseline Comparison": the chord of
every interval within r).  When the union of the column's own row (V0) is
one interval and the chords reaching L and U overlap it, the three chain and
the result is exactly [L, U].  Every other column goes to the general
kernels.  Each case is checked bit-exact against the oracle's float32 model,
within tolerance of the float64 oracle, and bit-exact against the same call
with DEXEL_FLAG_GENERAL (general kernels for every column).

The cases: solid slabs (every column settled by the test), balls, soups and
gyroid crops with many intervals per column (most columns general), grids
cut raggedly by the 64 x 16 tiles, and columns built so that one condition
fails: a far point reaching L whose chord stops short of V0 (at the rim of
the stencil, where the half-width is zero), a V0 of two intervals, an empty
row.
"""
from __future__ import annotations

import numpy as np
import pytest

from synth import gen
from tests.helpers import grid_from_columns
from tests.test_gpu_thin import _rng, check, slab_grid, thin_grid

pytestmark = pytest.mark.gpu


@pytest.mark.parametrize("nx,ny", [(1, 1), (1, 40), (70, 1), (64, 16), (65, 17), (131, 45)])
@pytest.mark.parametrize("r", [0.0, 1.5, 4.0, 11.5])
def test_solid_slabs(engine, oracle_lib, nx, ny, r):
    g = slab_grid(_rng("solid-slab", nx, ny, r), nx, ny, 10.0, 60.0, 8.0)
    cp = check(engine, oracle_lib, g, r, "dilate", "solid slab")
    assert np.diff(cp).max() == 1


@pytest.mark.parametrize("seed", [0, 3])
@pytest.mark.parametrize("r", [2.0, 3.0, 7.5, 16.0, 25.0])
def test_solid_spheres(engine, oracle_lib, seed, r):
    check(engine, oracle_lib, gen.spheres_grid(seed), r, "dilate", f"spheres seed{seed}")


@pytest.mark.parametrize("r", [1.0, 4.0, 16.0])
def test_solid_thin_and_thick(engine, oracle_lib, r):
    g = thin_grid(_rng("solid-mixed", r), 140, 70, 80.0, p_empty=0.2, p_thick=0.3, max_thick=5)
    check(engine, oracle_lib, g, r, "dilate", "mixed")


@pytest.mark.parametrize("r", [2.0, 6.0, 16.0])
def test_solid_gyroid_crop(engine, oracle_lib, r):
    g = gen.gyroid_grid(1, n=96, height=200.0, period=32.0)
    check(engine, oracle_lib, g, r, "dilate", "gyroid96")


@pytest.mark.parametrize("op", ["close", "open"])
def test_solid_chains(engine, oracle_lib, op):
    g = thin_grid(_rng("solid-chain", op), 100, 60, 40.0, p_empty=0.05, p_thick=0.2)
    check(engine, oracle_lib, g, 3.5, op, f"chain {op}")


def test_solid_conditions_fail(engine, oracle_lib):
    """Columns where the chaining fails: a point at depth -100 at the rim of
    the stencil (chord of zero half-width, so L = -100 and its chord ends at
    -100, far below V0), a row whose V0 has two intervals, an empty row."""
    nx, ny, r = 40, 30, 5.0
    cols = [[(0.0, 10.0)] for _ in range(nx * ny)]
    cols[12 * nx + 20] = [(-100.0, -100.0), (0.0, 10.0)]   # rim point for (20, 17) and (25, 12)
    for x in range(nx):
        cols[5 * nx + x] = [(0.0, 2.0), (40.0, 42.0)]      # V0 of row 5: two intervals
        cols[25 * nx + x] = []                             # empty row
    g = grid_from_columns(nx, ny, cols)
    cp = check(engine, oracle_lib, g, r, "dilate", "conditions")
    assert np.diff(cp)[17 * nx + 20] == 2  # the far point stays apart


def test_solid_batch(engine, oracle_lib):
    import paper_1804_08968_amd as dx
    rng = _rng("solid-batch")
    grids = [slab_grid(rng, 70, 20, 0.0, 30.0, 3.0), thin_grid(rng, 33, 65, 30.0, p_thick=0.4),
             gen.spheres_grid(2), slab_grid(rng, 1, 1, 0.0, 5.0, 1.0), thin_grid(rng, 129, 17, 30.0)]
    radii = [2.0, 3.5, 4.0, 1.0, 24.0]
    ops = ["dilate", "erode", "close", "dilate", "open"]
    dgs = [dx.DeviceGrid.from_host(g) for g in grids]
    print("[case] solid batch", flush=True)
    outs = dx.batch_offset(engine, dgs, radii, ops)
    for g, r, op, o in zip(grids, radii, ops, outs):
        col_ptr, z = o.to_host()
        ref = oracle_lib.run(g, r, op, "f32model")
        assert np.array_equal(col_ptr, ref.col_ptr), (op, r)
        assert np.array_equal(z[: 2 * col_ptr[-1]].astype(np.float64), ref.z), (op, r)
