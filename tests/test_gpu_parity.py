"""GPU parity: libdexel (through the C ABI) against the oracle.

Two bars for every case:
* bit-exact against the oracle's float32 model (same chord definition with
  one float32 rounding per end and a float32 half-width table): the GPU
  result is the float32 union of those chords whatever the order or pruning
  of its work, so column pointers and endpoints must be identical;
* within tolerance of the float64 oracle: endpoints within
  tau = max(1e-5, ulp32(|z| + r)) and segment counts equal except where a
  gap or interval is shorter than gamma = max(1e-6, 2 ulp32(|z| + r)).
"""
from __future__ import annotations

import zlib

import numpy as np
import pytest

from synth import gen
from tests.helpers import compare_columns, grid_from_columns, random_grid

pytestmark = pytest.mark.gpu


def gpu_run(engine, g, r, op):
    import paper_1804_08968_amd as dx
    dg = dx.DeviceGrid.from_host(g)
    out = engine.offset(dg, r, op)
    return out.to_host()


def check(engine, oracle, g, r, op, cols=None, label=""):
    print(f"[case] {label} nx={g.nx} ny={g.ny} nseg={g.nseg} r={r} op={op}", flush=True)
    col_ptr, z = gpu_run(engine, g, r, op)
    z = z.astype(np.float64)
    gcnt = np.diff(col_ptr)
    k = 2 if op in ("open", "close") else 1
    if cols is None:
        ref32 = oracle.run(g, r, op, "f32model")
        assert np.array_equal(col_ptr, ref32.col_ptr), "segment counts differ from float32 model"
        assert np.array_equal(z, ref32.z), "endpoints differ from float32 model"
        ref = oracle.run(g, r, op, "f64")
        res = compare_columns(np.diff(ref.col_ptr), ref.z, gcnt, z, r, k=k)
    else:
        cols = np.asarray(cols, dtype=np.int64)
        if op in ("dilate", "erode"):
            c32, z32 = oracle.offset_columns(g, r, op, "f32model", cols=cols)
            c64, z64 = oracle.offset_columns(g, r, op, "f64", cols=cols)
        else:
            c32, z32 = oracle.region_chain(g, r, op, cols, "f32model")
            c64, z64 = oracle.region_chain(g, r, op, cols, "f64")
        sel_cnt = gcnt[cols]
        sel_z = np.concatenate([z[2 * col_ptr[c]: 2 * col_ptr[c + 1]] for c in cols])
        assert np.array_equal(sel_cnt, c32)
        assert np.array_equal(sel_z, z32)
        res = compare_columns(c64, z64, sel_cnt, sel_z, r, k=k)
    assert res["failed"] == 0, res
    return res


@pytest.mark.parametrize("seed", range(10))
def test_c1_spheres(engine, oracle_lib, seed):
    g = gen.config_grid("c1", seed)
    check(engine, oracle_lib, g, 3.0, "dilate", label=f"c1 seed{seed}")


EDGE = [  # (label, nx, ny, height, r)
    ("ragged", 67, 13, 40.0, 2.5), ("row", 150, 1, 30.0, 3.0), ("column", 1, 90, 30.0, 2.0),
    ("tiny", 3, 2, 10.0, 4.0), ("r0", 33, 9, 20.0, 0.0), ("rhalf", 40, 21, 20.0, 0.5),
    ("r_sqrt2", 31, 17, 25.0, 1.41421356), ("wide_r", 19, 23, 30.0, 7.25),
]


@pytest.mark.parametrize("op", ["dilate", "erode", "close", "open"])
@pytest.mark.parametrize("label,nx,ny,height,r", EDGE)
def test_edge_shapes(engine, oracle_lib, label, nx, ny, height, r, op):
    rng = np.random.default_rng(zlib.crc32(f"{label}/{op}".encode()))
    g = random_grid(rng, nx, ny, height, max_per_col=4, p_empty=0.3)
    check(engine, oracle_lib, g, r, op, label=label)


def test_empty_grid(engine, oracle_lib):
    g = grid_from_columns(70, 5, [[] for _ in range(350)])
    check(engine, oracle_lib, g, 3.0, "dilate", label="empty")
    check(engine, oracle_lib, g, 3.0, "erode", label="empty")


def test_single_column(engine, oracle_lib):
    g = grid_from_columns(1, 1, [[(0.0, 5.0), (10.0, 11.5)]])
    for op in ("dilate", "erode", "close", "open"):
        check(engine, oracle_lib, g, 1.0, op, label="1x1")


def test_dense_columns_fallback(engine, oracle_lib):
    """Many short intervals per column: per-lane lists overflow LDS and the
    global-memory replay takes over."""
    rng = np.random.default_rng(5)
    cols = []
    for _ in range(48 * 10):
        k = int(rng.integers(40, 90))
        pts = np.sort(rng.uniform(0, 2000, 2 * k)).astype(np.float32).astype(np.float64)
        iv = [(pts[2 * i], pts[2 * i + 1]) for i in range(k) if pts[2 * i + 1] > pts[2 * i]]
        m = []
        for a, b in iv:
            if m and a <= m[-1][1]:
                m[-1] = (m[-1][0], max(b, m[-1][1]))
            else:
                m.append((a, b))
        cols.append(m)
    g = grid_from_columns(48, 10, cols)
    for op in ("dilate", "erode"):
        check(engine, oracle_lib, g, 2.0, op, label="dense")


def test_long_lists_grow_the_arena(engine, oracle_lib):
    """About 1500 short, well separated intervals per column: the row unions
    hold 1500 and more intervals, past every LDS list and past the arena
    tier's first lists, which then grow (256, 1024, 4096 entries) up to the
    column's bound.  The default workspace is too small for that arena, so
    the engine's retry from the reported need is exercised too."""
    rng = np.random.default_rng(11)
    nx, ny = 8, 4
    cols = []
    for _ in range(nx * ny):
        base = 10.0 * np.arange(1500) + rng.uniform(0.0, 3.0, 1500)
        a = base.astype(np.float32).astype(np.float64)
        b = (base + 0.5).astype(np.float32).astype(np.float64)
        cols.append(list(zip(a, b)))
    g = grid_from_columns(nx, ny, cols)
    for op in ("dilate", "erode", "close"):
        check(engine, oracle_lib, g, 1.5, op, label="long lists")


@pytest.mark.parametrize("r", [2.0, 8.0])
@pytest.mark.parametrize("op", ["dilate", "erode"])
def test_c2_full(engine, oracle_lib, r, op):
    g = gen.config_grid("c2", 0)
    check(engine, oracle_lib, g, r, op, label="c2")


@pytest.mark.parametrize("r", [2.0, 8.0])
@pytest.mark.parametrize("op", ["dilate", "erode"])
def test_c2lit_full(engine, oracle_lib, r, op):
    """The literal 200-primitive version of the 512^2 soup (about 0.8
    intervals per column), full grid."""
    g = gen.config_grid("c2lit", 0)
    check(engine, oracle_lib, g, r, op, label="c2lit")


@pytest.mark.parametrize("op", ["dilate", "erode"])
def test_c2lit_r32_sampled(engine, oracle_lib, op):
    g = gen.config_grid("c2lit", 1)
    rng = np.random.default_rng(10)
    cols = np.unique(np.concatenate([rng.integers(0, g.nx * g.ny, 1500),
                                     np.arange(0, 64), np.arange(g.nx * g.ny - 64, g.nx * g.ny)]))
    check(engine, oracle_lib, g, 32.0, op, cols=cols, label="c2lit r32")


@pytest.mark.parametrize("op", ["dilate", "erode"])
def test_c2_r32_sampled(engine, oracle_lib, op):
    g = gen.config_grid("c2", 1)
    rng = np.random.default_rng(9)
    cols = np.unique(np.concatenate([rng.integers(0, g.nx * g.ny, 1500),
                                     np.arange(0, 64), np.arange(g.nx * g.ny - 64, g.nx * g.ny)]))
    check(engine, oracle_lib, g, 32.0, op, cols=cols, label="c2 r32")


def test_gyroid_small_close(engine, oracle_lib):
    g = gen.gyroid_grid(0, n=128, height=256.0)
    check(engine, oracle_lib, g, 16.0, "close", label="gyroid128 close")


@pytest.mark.parametrize("op", ["dilate", "erode", "close"])
def test_slices_2d(engine, oracle_lib, op):
    """2D offsets of many slices (nx x 1 grids, Sec. 3.2) in one batched
    enqueue, each bit-exact against the oracle's float32 model of that slice
    and within tolerance of FP64."""
    rng = np.random.default_rng(21)
    hosts = []
    for k in range(24):
        nx = int(rng.integers(1, 300))
        hosts.append(random_grid(rng, nx, 1, 300.0, max_per_col=6, p_empty=0.3))
    import paper_1804_08968_amd as dx
    r = 6.5
    print(f"[case] slices {op} r={r} n={len(hosts)}", flush=True)
    outs = engine.offset_slices([dx.DeviceGrid.from_host(h) for h in hosts], r, op)
    k = 2 if op in ("open", "close") else 1
    for h, o in zip(hosts, outs):
        col, z = o.to_host()
        z = z.astype(np.float64)
        ref32 = oracle_lib.run(h, r, op, "f32model")
        assert np.array_equal(col, ref32.col_ptr)
        assert np.array_equal(z, ref32.z)
        ref = oracle_lib.run(h, r, op, "f64")
        res = compare_columns(np.diff(ref.col_ptr), ref.z, np.diff(col), z, r, k=k)
        assert res["failed"] == 0, res
