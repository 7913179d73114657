"""Erosion of thin columns (at most one interval in every column of the
ball's stencil): the tiled max / min filter against the oracle and against
the general kernels.

When each stencil column of an output column holds at most one interval,
the complement of each is two rays (the whole line if empty), so the union
of the complement's chords is (-inf, MA] U [MB, +inf) and the eroded column
is [MA, MB] or empty (Sec. 3.1, "Erosion", with the chords of Sec. 4,
"Baseline Comparison").  The library evaluates those columns with its own
kernel and leaves every other column to the general kernels, which then run
only where such a column needs them.  Each case is checked three ways:
bit-exact against the oracle's float32 model, within tolerance of the
float64 oracle, and bit-exact against the same call with DEXEL_FLAG_GENERAL
(general kernels for every column).

Grids cut the 64 x 16 tiles raggedly, mix in columns of two or more
intervals (alone, in clusters, at the grid border), hold empty columns, and
span radii from 0 to past the largest the tiled kernel takes (R = 32 needs
more LDS than one workgroup is given, so it runs on the general kernels).
"""
from __future__ import annotations

import zlib

import numpy as np
import pytest

from tests.helpers import compare_columns, grid_from_columns

pytestmark = pytest.mark.gpu


def thin_grid(rng, nx, ny, height, p_empty=0.05, p_thick=0.0, max_thick=4, clusters=0):
    """One interval per column (float32 endpoints), some empty; a fraction
    p_thick of the columns, and `clusters` 3 x 3 blocks, hold 2..max_thick."""
    n = nx * ny
    thick = rng.random(n) < p_thick
    for _ in range(clusters):
        cx, cy = int(rng.integers(0, nx)), int(rng.integers(0, ny))
        for yy in range(max(0, cy - 1), min(ny, cy + 2)):
            for xx in range(max(0, cx - 1), min(nx, cx + 2)):
                thick[yy * nx + xx] = True
    cols = []
    for c in range(n):
        if rng.random() < p_empty:
            cols.append([])
            continue
        k = int(rng.integers(2, max_thick + 1)) if thick[c] else 1
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


def slab_grid(rng, nx, ny, lo, hi, jitter):
    """Every column one interval [lo + u, hi - v], u, v ~ U[0, jitter]."""
    cols = []
    for _ in range(nx * ny):
        a = np.float64(np.float32(lo + rng.uniform(0, jitter)))
        b = np.float64(np.float32(hi - rng.uniform(0, jitter)))
        cols.append([(a, b)])
    return grid_from_columns(nx, ny, cols)


def run(engine, g, r, op, flags=0):
    import paper_1804_08968_amd as dx
    dg = dx.DeviceGrid.from_host(g)
    col_ptr, z = engine.offset(dg, r, op, flags=flags).to_host()
    return col_ptr, z.astype(np.float64)


def check(engine, oracle, g, r, op, label):
    import paper_1804_08968_amd as dx
    print(f"[case] thin {label} nx={g.nx} ny={g.ny} nseg={g.nseg} r={r} op={op}", flush=True)
    col_ptr, z = run(engine, g, r, op)
    gcp, gz = run(engine, g, r, op, flags=dx.DEXEL_FLAG_GENERAL)
    assert np.array_equal(col_ptr, gcp), "counts differ from the general kernels"
    assert np.array_equal(z[: 2 * col_ptr[-1]], gz[: 2 * gcp[-1]]), "endpoints differ from the general kernels"
    ref32 = oracle.run(g, r, op, "f32model")
    assert np.array_equal(col_ptr, ref32.col_ptr), "counts differ from the float32 model"
    assert np.array_equal(z[: 2 * col_ptr[-1]], ref32.z), "endpoints differ from the float32 model"
    ref = oracle.run(g, r, op, "f64")
    res = compare_columns(np.diff(ref.col_ptr), ref.z, np.diff(col_ptr), z[: 2 * col_ptr[-1]], r,
                          k=2 if op in ("open", "close") else 1)
    assert res["failed"] == 0, res
    return col_ptr


SIZES = [(1, 1), (1, 50), (90, 1), (64, 16), (65, 17), (130, 40), (257, 33)]
RADII = [0.0, 0.5, 1.5, 3.0, 7.25, 16.0, 24.5, 32.0]


def _rng(*key):
    return np.random.default_rng(zlib.crc32(repr(key).encode()))


@pytest.mark.parametrize("nx,ny", SIZES)
@pytest.mark.parametrize("r", [0.0, 1.5, 7.25, 24.5])
def test_thin_erosion_sizes(engine, oracle_lib, nx, ny, r):
    g = thin_grid(_rng("sizes", nx, ny, r), nx, ny, 40.0, p_empty=0.02)
    check(engine, oracle_lib, g, r, "erode", "sizes")


@pytest.mark.parametrize("r", RADII)
def test_thin_erosion_radii(engine, oracle_lib, r):
    g = slab_grid(_rng("slab", r), 96, 70, 0.0, 120.0, 6.0)
    cp = check(engine, oracle_lib, g, r, "erode", "slab")
    if r <= 16.0:
        assert np.diff(cp).min() == 1  # a slab thick enough stays one interval everywhere


@pytest.mark.parametrize("p_thick,clusters", [(0.002, 0), (0.0, 3), (0.05, 2), (0.5, 0), (1.0, 0)])
@pytest.mark.parametrize("r", [1.0, 3.0, 16.0])
def test_thin_erosion_mixed(engine, oracle_lib, p_thick, clusters, r):
    """Columns of several intervals among thin ones: the output columns whose
    stencil reaches them go to the general kernels, which run their stages
    only on the rows those columns need."""
    g = thin_grid(_rng("mixed", p_thick, clusters, r), 150, 90, 60.0, p_empty=0.03,
                  p_thick=p_thick, clusters=clusters)
    check(engine, oracle_lib, g, r, "erode", f"mixed p={p_thick} clusters={clusters}")


@pytest.mark.parametrize("op", ["close", "open"])
@pytest.mark.parametrize("r", [2.0, 5.5])
def test_thin_chains(engine, oracle_lib, op, r):
    """A closing's erosion reads the dilation's result (one interval per
    column where the dilation filled the gaps, more elsewhere); an opening's
    erosion reads thin input and its dilation the thin result."""
    rng = _rng("chain", op, r)
    if op == "close":
        g = thin_grid(rng, 120, 75, 50.0, p_empty=0.1, p_thick=0.3, max_thick=3)
    else:
        g = thin_grid(rng, 120, 75, 50.0, p_empty=0.02, clusters=2)
    check(engine, oracle_lib, g, r, op, "chain")


def test_thin_in_batch(engine, oracle_lib):
    """Thin erosions among dilations and general erosions in one batch: the
    tiles of the thin items are numbered across the batch."""
    import paper_1804_08968_amd as dx
    rng = _rng("batch")
    grids = [thin_grid(rng, 70, 20, 30.0), thin_grid(rng, 33, 65, 30.0, p_thick=0.4),
             thin_grid(rng, 64, 64, 30.0, p_thick=0.01), thin_grid(rng, 1, 1, 30.0),
             thin_grid(rng, 129, 17, 30.0)]
    radii = [2.0, 3.5, 4.0, 1.0, 24.0]
    ops = ["erode", "dilate", "close", "erode", "open"]
    dgs = [dx.DeviceGrid.from_host(g) for g in grids]
    print("[case] thin batch", flush=True)
    outs = dx.batch_offset(engine, dgs, radii, ops)
    for g, r, op, o in zip(grids, radii, ops, outs):
        col_ptr, z = o.to_host()
        ref = oracle_lib.run(g, r, op, "f32model")
        assert np.array_equal(col_ptr, ref.col_ptr), (op, r)
        assert np.array_equal(z[: 2 * col_ptr[-1]].astype(np.float64), ref.z), (op, r)
