"""GPU parity of dexel_dexelize (balls and boxes along cell-centre rays),
through the C ABI.

Chord ends are float64 operations rounded once each and then rounded once to
float32 on both sides, so the bar is bit-exact: against the oracle
(oracle/dexelize.py) on grids it finishes in seconds, and against the
workload generator (which the CPU pins tie to the oracle) at full size.
"""
from __future__ import annotations

import math

import numpy as np
import pytest
import torch

from oracle import dexelize as od
from synth import gen

pytestmark = pytest.mark.gpu


def _dx():
    import paper_1804_08968_amd as dx
    return dx


def run(engine, nx, ny, prims):
    col, z = engine.dexelize(nx, ny, np.asarray(prims, dtype=np.float64).reshape(-1, 7)).to_host()
    return col, z.astype(np.float64)


def random_prims(rng, n, count, smax):
    prims = []
    for _ in range(count):
        if rng.random() < 0.5:
            prims.append((od.BALL, *rng.uniform(-2, n + 2, 3), rng.uniform(0.3, smax), 0.0, 0.0))
        else:
            lo = rng.uniform(-2, n + 2, 3)
            prims.append((od.BOX, *lo, *(lo + rng.uniform(0.0, 2 * smax, 3))))
    return prims


@pytest.mark.parametrize("seed", range(4))
def test_random_sets(engine, seed):
    """Several 64-column tiles with a ragged tail; footprints cross the border."""
    rng = np.random.default_rng(seed)
    nx, ny = 45, 23
    prims = random_prims(rng, max(nx, ny), 40, 6.0)
    print(f"[case] dexelize random seed {seed}", flush=True)
    col, z = run(engine, nx, ny, prims)
    rc, rz = od.dexelize(nx, ny, prims)
    assert np.array_equal(col, rc)
    assert np.array_equal(z, rz)


@pytest.mark.parametrize("nx,ny,count", [(130, 9, 700), (300, 1, 600), (70, 3, 300), (257, 5, 513)])
def test_tiles_and_chunks(engine, nx, ny, count):
    """Grids that cut the kernel's cell tiles (64 x 4, or 256 x 1 below 4
    rows) raggedly, and lists of several primitive chunks with a ragged last
    one."""
    rng = np.random.default_rng(nx * 1000 + ny)
    prims = []
    for _ in range(count):   # centres and corners spread over this grid's own extent
        x0, y0, z0 = rng.uniform(-2, nx + 2), rng.uniform(-2, ny + 2), rng.uniform(0, 40)
        if rng.random() < 0.5:
            prims.append((od.BALL, x0, y0, z0, rng.uniform(0.3, 5.0), 0.0, 0.0))
        else:
            prims.append((od.BOX, x0, y0, z0, *(np.array([x0, y0, z0]) + rng.uniform(0.0, 10.0, 3))))
    print(f"[case] dexelize tiles {nx}x{ny} with {count} primitives", flush=True)
    col, z = run(engine, nx, ny, prims)
    rc, rz = od.dexelize(nx, ny, prims)
    assert np.array_equal(col, rc)
    assert np.array_equal(z, rz)


def test_culling_at_tile_edges(engine):
    """Primitives centred in one cell tile that reach the nearest cell centre
    of the next tile by a hair, or miss it by a hair: balls 1.25 from that
    centre with radius 1.25 +- 2^-40 across the x edge (columns 63 | 64) and
    the y edge (rows 3 | 4), and boxes whose high x corner is 64.5 +- 2^-40
    (column 64's centre)."""
    eps = 2.0 ** -40
    prims = []
    for k in range(12):
        cz, r = 4.0 * k, 1.25 + (eps if k % 2 else -eps)
        prims.append((od.BALL, 64.75, 1.5 + k % 3, cz, r, 0.0, 0.0))    # reaches column 63?
        prims.append((od.BALL, 63.25, 5.5 + k % 3, cz, r, 0.0, 0.0))    # reaches column 64?
        prims.append((od.BALL, 10.5 + k, 4.75, cz, r, 0.0, 0.0))        # reaches row 3?
        prims.append((od.BOX, 60.0 + k % 3, 3.0 + k % 2, cz, 64.5 + (eps if k % 2 else -eps), 4.5, cz + 1.0))
    print("[case] dexelize culling at tile edges", flush=True)
    col, z = run(engine, 130, 9, prims)
    rc, rz = od.dexelize(130, 9, prims)
    assert np.array_equal(col, rc)
    assert np.array_equal(z, rz)
    # the hair decides: the balls of odd k reach across the edge, those of even k do not
    def ncol(x, y):
        return int(rc[y * 130 + x + 1] - rc[y * 130 + x])
    assert [ncol(63, y) for y in (1, 2)] == [2, 2]
    assert [ncol(64, y) for y in (5, 6, 7)] == [2, 2, 2]
    assert [ncol(10 + k, 3) for k in range(12)] == [k % 2 for k in range(12)]


def test_deep_columns_beside_shallow_ones(engine):
    """A stack of 30 thin boxes over a few cells among random primitives: the
    cell tiles holding those columns need more list slots than the others
    (they are redone at full capacity, neighbouring lanes included)."""
    rng = np.random.default_rng(5)
    nx, ny = 200, 11
    prims = [(od.BALL, rng.uniform(0, nx), rng.uniform(0, ny), rng.uniform(0, 300), rng.uniform(0.5, 4.0), 0, 0)
             for _ in range(300)]
    prims += [(od.BOX, 60.0, 3.0, 10.0 * k, 70.0, 6.0, 10.0 * k + 2.0) for k in range(30)]
    prims += [(od.BOX, 190.0, 9.0, 7.0 * k, 200.0, 11.0, 7.0 * k + 3.0) for k in range(40)]
    print("[case] dexelize deep columns", flush=True)
    col, z = run(engine, nx, ny, prims)
    rc, rz = od.dexelize(nx, ny, prims)
    assert int(np.max(np.diff(rc))) > 30
    assert np.array_equal(col, rc)
    assert np.array_equal(z, rz)


@pytest.mark.parametrize("axis", ["x", "y"])
@pytest.mark.parametrize("seed", range(2))
def test_rays_along_x_and_y(engine, axis, seed):
    """Rays along x (grid over y, z) and along y (grid over z, x) on a box of
    unequal sides, so that a swapped grid axis cannot pass."""
    rng = np.random.default_rng(40 + seed)
    ext = np.array([70.0, 45.0, 30.0])
    prims = []
    for _ in range(400):
        c = rng.uniform(-2, ext + 2)
        if rng.random() < 0.5:
            prims.append((od.BALL, *c, rng.uniform(0.5, 6.0), 0.0, 0.0))
        else:
            prims.append((od.BOX, *c, *(c + rng.uniform(0.0, 9.0, 3))))
    nu, nv = {"x": (45, 30), "y": (30, 70)}[axis]
    print(f"[case] dexelize rays along {axis} seed {seed}", flush=True)
    col, z = engine.dexelize(nu, nv, np.asarray(prims), axis=axis).to_host()
    rc, rz = od.dexelize(nu, nv, prims, axis=axis)
    assert np.array_equal(col, rc)
    assert np.array_equal(z.astype(np.float64), rz)


def test_exact_boundaries(engine):
    """A ball whose radius reaches a neighbouring cell centre exactly (excluded:
    the lateral test is strict), a box whose edges pass through cell centres
    (included), a zero-height box, touching and overlapping chords."""
    prims = [
        (od.BALL, 2.5, 2.5, 0.0, 1.0, 0.0, 0.0),
        (od.BOX, 4.5, 0.5, 3.0, 6.5, 1.5, 4.0),
        (od.BOX, 0.5, 4.5, 7.0, 0.5, 4.5, 7.0),
        (od.BOX, 4.5, 0.5, 4.0, 4.5, 0.5, 5.0),
        (od.BALL, 5.5, 0.5, 6.0, 2.0, 0.0, 0.0),
    ]
    print("[case] dexelize boundaries", flush=True)
    col, z = run(engine, 8, 6, prims)
    rc, rz = od.dexelize(8, 6, prims)
    assert np.array_equal(col, rc)
    assert np.array_equal(z, rz)
    # the ball's only column is its own cell
    c = 2 * 8 + 2
    assert col[c + 1] - col[c] == 1 and list(z[2 * col[c]: 2 * col[c] + 2]) == [-1.0, 1.0]


def test_empty(engine):
    col, z = run(engine, 5, 3, np.zeros((0, 7)))
    assert col.tolist() == [0] * 16


def test_soup_full_size_equals_generator(engine):
    """The 512^2 soup of 1350 primitives, built on the GPU, equals the
    workload generator's grid bit for bit."""
    rec = gen.primitive_records(0)
    g = gen.primitives_grid(0)
    print("[case] dexelize c2 soup", flush=True)
    col, z = run(engine, 512, 512, rec)
    assert np.array_equal(col, g.col_ptr)
    assert np.array_equal(z, np.asarray(g.z, dtype=np.float64).reshape(-1))


@pytest.mark.parametrize("i", [0, 7, 21])
def test_batch_shapes_equal_generator(engine, i):
    rng = np.random.default_rng(0)
    for k in range(i + 1):   # the draws of batch_shapes(0), shape by shape
        s = int(round(math.exp(rng.uniform(math.log(128), math.log(1024)))))
        nprim = int(rng.integers(20, 301))
        rng.uniform(2.0, 32.0)
        sub = int(rng.integers(0, 2**31 - 1))
    scale = s / 512.0
    kw = dict(n=s, count=nprim, smin=4.0 * scale, smax=64.0 * scale, height=float(s))
    g = gen.primitives_grid(sub, **kw)
    print(f"[case] dexelize batch shape {i} side {s}", flush=True)
    col, z = run(engine, s, s, gen.primitive_records(sub, **kw))
    assert np.array_equal(col, g.col_ptr)
    assert np.array_equal(z, np.asarray(g.z, dtype=np.float64).reshape(-1))


def test_errors_reported(engine):
    dx = _dx()
    print("[case] dexelize errors", flush=True)
    with pytest.raises(dx.DexelError) as e:   # both ray axes at once
        ws = torch.empty(dx.dexel_dexelize_workspace_size(engine.ctx, 4, 4), dtype=torch.uint8, device="cuda")
        o = (torch.empty(17, dtype=torch.int64, device="cuda"), torch.empty(64, dtype=torch.float32, device="cuda"),
             torch.zeros(1, dtype=torch.int64, device="cuda"), torch.zeros(1, dtype=torch.int32, device="cuda"))
        p = torch.zeros((1, 7), dtype=torch.float64, device="cuda")
        st = dx.dexel_dexelize(engine.ctx, 4, 4, p, dx.make_out(4, 4, *o), ws, None,
                               dx.DEXEL_FLAG_SYNC | dx.DEXEL_FLAG_RAYS_X | dx.DEXEL_FLAG_RAYS_Y)
        raise dx.DexelError(st, "")
    assert e.value.status == dx.DEXEL_ERR_INVALID
    with pytest.raises(dx.DexelError) as e:
        engine.dexelize(4, 4, [(7.0, 0, 0, 0, 1, 1, 1)])
    assert e.value.status == dx.DEXEL_ERR_INVALID
    # 70 separated boxes on one column: more than a column may hold
    boxes = [(od.BOX, 0.0, 0.0, 10.0 * k, 1.0, 1.0, 10.0 * k + 1.0) for k in range(70)]
    with pytest.raises(dx.DexelError) as e:
        engine.dexelize(2, 2, boxes)
    assert e.value.status == dx.DEXEL_ERR_UNSUPPORTED
    # 60 fit; the engine retries past a small first capacity
    boxes = [(od.BOX, 0.0, 0.0, 10.0 * k, 40.0, 40.0, 10.0 * k + 1.0) for k in range(60)]
    col, z = run(engine, 40, 40, boxes)
    rc, rz = od.dexelize(40, 40, boxes)
    assert np.array_equal(col, rc) and np.array_equal(z, rz)
